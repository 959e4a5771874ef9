// Host-side launchers of the libtcol kernels (one per kernel family).
#pragma once

#include "tcol_internal.h"

namespace tcol {

// initial weights N(0, sigma0^2) from Philox4x32-10 (stream 1) and Box-Muller
hipError_t launch_init_weights(float* W, long long count, unsigned long long seed, double sigma0, hipStream_t s);
// validates A, writes A8 and the operand copy, adds the number of ones of A to *ones
hipError_t launch_pack_graph(const uint8_t* A, int n, int n_pad, int prec, uint8_t* A8, void* Aop, int* bad,
                             unsigned long long* ones, hipStream_t s);
hipError_t launch_colors(const GraphDev* gd, int G, int total_rows, int honor_stop, hipStream_t s);
// class sizes and vertex-major colours; with lists != 0 also the class lists of graphs on the
// sparse penalty (dynamic LDS from prep_lds)
size_t prep_lds(int kmax, int nmax, int lists);
// decide: graphs on the sparse rows also take the iteration's penalty choice (pdense);
// ex_blocks > 0: the same launch also runs the expansion's blocks (as launch_expand with
// gate 1 and the same honor_stop and next), which must then not depend on the choice;
// advance_prev: the launch first ends the previous iteration (as launch_advance)
hipError_t launch_prep(const GraphDev* gd, int G, int total_mem, size_t lds, int honor_stop, int next, int decide,
                       int ex_blocks, int advance_prev, hipStream_t s);
hipError_t penalty_sparse_prepare();
// sparse penalty rows: one row per block of `threads` (256, 512 or 1024), members PM = 8 at a
// time
size_t penalty_sparse_lds(int PM, int kmax, int dmax, int nmax);
// accumulate 0: rows written to G before the contraction (epilogue path); 1: added to the
// contraction's G (fast path).
// kw > 0 (penalty_sparse_kw of the largest k of those graphs; PM at most threads / 64): graphs
// with pfuse take their row update in this launch as well, in every iteration (accumulate 1);
// add: some such graph has an added fitness term (equity or colour cost)
hipError_t launch_penalty_sparse(const GraphDev* gd, int G, int blocks, int PM, int threads, int kw, int add,
                                 size_t lds, int honor_stop, int accumulate, hipStream_t s);
// values per lane of the fused row update for k <= kmax (2, 3, 5, 7 or 9), or -1 past k = 576
int penalty_sparse_kw(int kmax);
hipError_t launch_expand(const GraphDev* gd, int G, int total_blocks, int honor_stop, int next, int gate,
                         hipStream_t s);
hipError_t launch_mtilde(const GraphDev* gd, int G, int total_tiles, int honor_stop, int flags, int gsel,
                         int32_t* mt_out, hipStream_t s);
hipError_t launch_fitness(const GraphDev* gd, int G, int honor_stop, int flags, int gsel, hipStream_t s);
hipError_t launch_update(const GraphDev* gd, int G, int total_rows, int honor_stop, int mode, int gsel,
                         float* gS_out, float* gW_out, hipStream_t s);
// register-resident row update for k <= 576 (update_rows_kpl(kmax) != 0); mode 0 also colours the new rows
int update_rows_kpl(int kmax);
// var: bit 0 some graph has an added fitness term, bit 1 some graph takes heavy-ball steps
hipError_t launch_update_rows(const GraphDev* gd, int G, int total_rows, int kmax, int var, int honor_stop, int mode,
                              int gsel, float* gS_out, float* gW_out, hipStream_t s);
hipError_t launch_advance(const GraphDev* gd, int G, hipStream_t s);
hipError_t launch_loss(const GraphDev* gd, int g, int ntiles, double* out, hipStream_t s);
hipError_t launch_copy_report(const GraphDev* gd, int g, int16_t* colors, int64_t* fcol, int64_t* feq,
                              hipStream_t s);
// graph g's selection as [d][i][s] (s < cmax), -1 past a vertex's demand
hipError_t launch_copy_selection(const GraphDev* gd, int g, int16_t* out, hipStream_t s);
hipError_t launch_state(const GraphDev* gd, int G, int op, int g_only, long long t, hipStream_t s);
// class-conflict matrices S_d^T (A.S_d) of graph g ([D][k][k] int32) from G = A.S and the colours
hipError_t launch_class_conflicts(const GraphDev* gd, int g, int D, int k, int32_t* out, hipStream_t s);
// one graph's descriptor and a fresh state written on the device from kernel arguments
hipError_t launch_put_desc(const GraphDev& d, GraphDev* gd, GraphState* st, hipStream_t s);
// bytes (a multiple of 16) of 16-byte aligned device memory set to zero by a kernel
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

// MFMA contraction G = A.S (+ P.S) with the conflict gather.
//   mode 0: store G [D][n][k] (separate-kernel path); 1: fused softmax/update/argmax epilogue
//   passes: bit 0 = A.S with gather, bit 1 = penalty pass when active, bit 2 = store / epilogue,
//           bit 3 = dense penalty operand even for graphs on the sparse penalty, bit 4 = no
//           penalty pass at all, bit 5 = A.S counts as uint16 for graphs whose sparse rows take
//           the row update (pfuse) in iterations on the sparse rows (mode 0; the fast path's step),
//           bit 6 = no f_color gather for graphs whose iteration takes
//           the sparse rows (the sparse kernel gathers it from G), bit 7 = no gather at all
struct GemmShape {
    int prec, bm, ntw, mode;
};
bool gemm_supported(const GemmShape& s);
hipError_t gemm_prepare(const GemmShape& s);       // sets the LDS attribute of the instantiation
hipError_t launch_gemm(const GemmShape& s, const GraphDev* gd, int G, int total_tiles, int honor_stop,
                       int passes, int cstage, hipStream_t st);
// dynamic LDS of a GEMM launch (cstage: bytes of member colours staged by the fused epilogue)
size_t gemm_lds_bytes(const GemmShape& s, int cstage);
int gemm_bn(int ntw);

// One launch for a run of iterations over all graphs (fast schedule, dense penalty
// pass, no heavy-ball steps, one operand precision): a queue of items in segments, one per
// (iteration, phase, graph) in that order, phases 0 class sizes + expansion, 1 group
// concentration, 2 contraction tiles, 3 fitness, 4 row update.  Segment s holds tickets
// [start, next start) of graph g; its items wait until `need` items of graph g are done.
struct BatchSeg {
    int start, g, phase, iter, need;
    int pad[3];
};
// contraction tile of the batch launch (rows per block, 16-column subtiles per wave), and the
// expansion blocks, group-concentration tiles and 16-row groups of the row update per item
constexpr int kBatchBM = 64, kBatchNTW = 4;
constexpr int kBatchExpand = 8, kBatchMtilde = 4, kBatchRowGroups = 8;
// control words before the per-graph done counts: [0] abort flag (cleared when tcol_step
// starts), [4] ticket and [5] tickets past the end (cleared before every launch)
constexpr int kBatchCtl = 8;
// the row update's values per 16-lane group (8 or 36; 0: k too large)
int batch_kpl(int kmax);
// dynamic LDS of the launch (prep_bytes: the class-size block's, prep_lds)
size_t batch_lds_bytes(int prec, size_t prep_bytes);
// LDS attribute; resident blocks per CU of the instantiation
hipError_t batch_prepare(int prec, int kpl, int* blocks_per_cu);
// nseg segments of `total` tickets; ctl: kBatchCtl + G ints, words 4.. zero at launch, word 0 the
// sticky abort flag; cancel: a word the host may set (device view of pinned host memory), read by
// waits and by every 256th item; spin_limit: polls of a wait before it gives up
hipError_t launch_batch_run(int prec, int kpl, int grid, size_t lds, const GraphDev* gd, int G, const BatchSeg* segs,
                            int nseg, int total, int* ctl, const int* cancel, int spin_limit, hipStream_t s);

}  // namespace tcol
