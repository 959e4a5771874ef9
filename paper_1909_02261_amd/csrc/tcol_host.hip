// Host runtime of libtcol: the C ABI declared in include/tcol.h.
//
// A context holds G graphs stepped together.  All device memory lives in one
// workspace (caller-provided or allocated here): a head with the descriptor
// and state arrays of all graphs, then one region per graph.  Each launch in a
// step covers every graph of the context through flattened work indices, and
// the step sequence is captured once into a hipGraph and replayed, since every
// kernel reads the iteration counter, the buffer parities and the stop flags
// from device memory.
//
// Three step sequences (tcol_options.fused):
//   0 plain: colours -> classes -> one-hot S -> dense penalty operand -> contraction
//     storing G -> fitness / stop -> update -> counter;
//   1 fast: classes -> penalty rows (sparse kernel) or dense operand -> one-hot S ->
//     contraction storing G -> fitness / stop -> update that also colours the new rows
//     -> counter (the colours of the first iteration come from one argmax pass);
//   2 epilogue: classes -> penalty -> one-hot S -> contraction whose epilogue updates W
//     into the second buffer and colours the result -> fitness / stop, which accepts
//     the update by flipping the buffers.
#include "tcol_internal.h"
#include "tcol_launch.h"
#include "../../include/tcol.h"

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace tcol;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxLdsBytes = 160 * 1024;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

enum Buf {
    B_LUT_PEN, B_LUT_BON, B_LUT_KA, B_LUT_VB, B_DEM, B_SEL, B_W2, B_A8, B_AOP, B_POP, B_S0, B_S1, B_SP0, B_SP1, B_C0, B_C1,
    B_V0, B_V1, B_G, B_F2, B_F2P, B_FCOL, B_FEQ, B_F, B_PART, B_SNAP, B_CT, B_CLSV, B_CLSOFF, B_CINFO, B_SQ, B_VEL, B_COUNT
};

struct Layout {
    size_t off[B_COUNT];
    size_t total;
    int n_pad, rows_S, mt_ts, mt_T, mt_tiles;
};


// colours per vertex of a graph (its multicolouring demands' maximum, else 1)
int cmax_of(const tcol_graph_params& p) { return p.problem == TCOL_MCOL ? std::max(1, (int)p.max_demand) : 1; }

Layout make_layout(const tcol_graph_params& p) {
    Layout L{};
    L.n_pad = round_up(p.n, kPadN);
    L.rows_S = round_up(p.D * p.k, 16) + kSRowSlack;
    // group-concentration tiles: 32 x 32 for small graphs (more blocks), else 64 x 64
    L.mt_ts = L.n_pad <= 2048 ? 32 : 64;
    L.mt_T = L.n_pad / L.mt_ts;
    L.mt_tiles = L.mt_T * (L.mt_T + 1) / 2;
    const size_t n2 = (size_t)L.n_pad * L.n_pad;
    const size_t dnk = (size_t)p.D * p.n * p.k;
    size_t sz[B_COUNT];
    // tables over the group concentration 0 .. D cmax (cmax colours per vertex: multicolouring)
    const int cm = cmax_of(p);
    const size_t nlut = (size_t)p.D * cm + 1;
    sz[B_LUT_PEN] = sizeof(float) * nlut;
    sz[B_LUT_BON] = sizeof(float) * nlut;
    sz[B_LUT_KA] = sizeof(double) * nlut;
    sz[B_LUT_VB] = sizeof(double) * nlut;
    sz[B_DEM] = sizeof(int32_t) * (size_t)p.n;
    sz[B_SEL] = cm > 1 ? sizeof(int16_t) * ((size_t)p.D * cm * round_up(p.n, 64) + 64) : 0;
    sz[B_W2] = sizeof(float) * dnk;
    sz[B_A8] = n2;
    sz[B_AOP] = (size_t)L.n_pad * op_row_bytes(p.precision, L.n_pad);
    sz[B_POP] = n2 * (p.precision == TCOL_FP32 ? 4 : 2);
    sz[B_S0] = sz[B_S1] = (size_t)L.rows_S * op_row_bytes(p.precision, L.n_pad);
    sz[B_SP0] = sz[B_SP1] = prec_split(p.precision) ? (size_t)L.rows_S * L.n_pad * 2 : 0;
    sz[B_C0] = sz[B_C1] = sizeof(int16_t) * ((size_t)p.D * round_up(p.n, 64) + 64);
    sz[B_V0] = sz[B_V1] = sizeof(int32_t) * (size_t)p.D * p.k;
    sz[B_G] = sizeof(float) * dnk;
    sz[B_F2] = sizeof(int32_t) * p.D;
    sz[B_F2P] = sizeof(int32_t) * (size_t)p.D * kF2Slots;
    sz[B_FCOL] = sz[B_FEQ] = sz[B_F] = sizeof(int64_t) * p.D;
    sz[B_PART] = sizeof(double) * 2 * (size_t)L.mt_tiles;
    sz[B_SNAP] = sizeof(int16_t) * (size_t)p.n * cm;
    sz[B_CT] = sizeof(int16_t) * (size_t)round_up(p.D, 8) * p.n;
    sz[B_CLSV] = sizeof(int16_t) * (size_t)p.D * round_up(p.n, 64);
    sz[B_CLSOFF] = sizeof(int32_t) * (size_t)p.D * (p.k + 1);
    sz[B_CINFO] = 8 * (size_t)p.D * round_up(p.n, 64);
    sz[B_SQ] = sizeof(long long) * (size_t)p.D;
    sz[B_VEL] = p.momentum != 0.0f ? sizeof(float) * dnk : 0;
    size_t o = 0;
    for (int b = 0; b < B_COUNT; ++b) {
        L.off[b] = o;
        o += align_up(sz[b]);
    }
    L.total = o;
    return L;
}

// runs of the batch launch: at most this many iterations (tcol_options.unroll's range)
constexpr int kBatchMaxIters = 64;
constexpr int kBatchPhases = 5;
size_t batch_ctl_bytes(int G) { return align_up(sizeof(int) * (kBatchCtl + (size_t)G)); }
size_t batch_seg_bytes(int G) { return align_up(sizeof(BatchSeg) * (size_t)kBatchMaxIters * kBatchPhases * G); }
// descriptors, states, the batch launch's control words and its item segments
size_t head_bytes(int G) {
    return align_up(sizeof(GraphDev) * G) + align_up(sizeof(GraphState) * G) + batch_ctl_bytes(G) + batch_seg_bytes(G);
}
// default polls of a wait in the batch launch before it gives up (each poll sleeps about 50 ns
// and reads device memory: seconds in all)
constexpr int kBatchSpinDefault = 1 << 22;

tcol_status check_params(const tcol_graph_params& p) {
    if (p.n < 1 || p.n > kMaxN || p.k < 1 || p.k > kMaxK || p.D < 1 || p.D > kMaxD) return TCOL_ESHAPE;
    if ((long long)p.D * p.k > (1LL << 26)) return TCOL_ESHAPE;
    if (p.problem < TCOL_KCOL || p.problem > TCOL_MCOL) return TCOL_EINVAL;
    if (p.problem == TCOL_MCOL) {
        if (p.max_demand < 1 || p.max_demand > kMaxDemand || p.max_demand > p.k) return TCOL_EINVAL;
        if (p.momentum != 0.0f) return TCOL_EINVAL;
        if (p.k > 1024) return TCOL_ESHAPE;
    } else if (p.max_demand < 0 || p.max_demand > 1) {
        return TCOL_EINVAL;
    }
    if (!(p.momentum >= 0.0f && p.momentum < 1.0f)) return TCOL_EINVAL;
    if (p.precision < TCOL_FP32 || p.precision > TCOL_FP4) return TCOL_EINVAL;
    if (!(p.eta > 0.0f) || !(p.rho >= 1.0f) || p.nb_iter < 1) return TCOL_EINVAL;
    if (!(p.lambda >= 0.0f) || !(p.mu >= 0.0f) || !(p.nu >= 0.0f)) return TCOL_EINVAL;
    if (p.lambda > 0.0f && !(p.alpha > 1.0f)) return TCOL_EINVAL;
    if (p.mu > 0.0f && !(p.beta > 1.0f)) return TCOL_EINVAL;
    if (!isfinite(p.alpha) || !isfinite(p.beta) || !isfinite(p.eta) || !isfinite(p.rho)) return TCOL_EINVAL;
    if (!isfinite(p.lambda) || !isfinite(p.mu) || !isfinite(p.nu)) return TCOL_EINVAL;
    return TCOL_OK;
}

double pow0(double x, double p) { return x == 0.0 ? 0.0 : pow(x, p); }

// shapes the contraction kernel is instantiated for: (rows per block, 16-column subtiles per wave)
const int kShapes[][2] = {{64, 2}, {64, 4}, {128, 4}, {128, 6}, {128, 8}, {64, 9}, {128, 9}, {256, 4}, {256, 6}};

}  // namespace

struct tcol_ctx {
    int G = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    std::vector<tcol_graph_params> params;
    std::vector<Layout> layouts;
    std::vector<GraphDev> hdesc;
    GraphDev* ddesc = nullptr;
    GraphState* dstate = nullptr;
    GraphState* hstate = nullptr;   // pinned
    uint8_t* ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_owned = false;
    tcol_options opt{};
    GemmShape shape{};              // separate-path tiling (also used by tcol_conflicts / tcol_loss_grad)
    GemmShape fshape{};             // fused-path tiling
    bool fused_ok = false;          // the fused path is available for these graphs
    bool any_momentum = false;      // some graph takes heavy-ball steps (no epilogue path)
    bool any_mcol = false;          // some graph is a multicolouring (plain path only)
    int update_var = 0;             // row-update variant: bit 0 added fitness term, bit 1 momentum
    int ps_PM = 0, ps_threads = 0;  // sparse penalty: members per accumulator group, block size
    int ps_kw = 0;                  // sparse penalty: values per lane of the fused row update (0: none)
    bool all_pfuse = false;         // every graph's row update rides on the sparse-rows launch
    // batch launch (fused = 3): one launch per run of iterations, items in segments
    bool batch_ok = false;
    int batch_kpl = 0, batch_grid_cap = 0, batch_prec = 0;
    int batch_items = 0;            // items of one iteration over all graphs
    size_t batch_lds = 0;
    int* dctl = nullptr;            // workspace: kBatchCtl + G ints
    BatchSeg* dsegs = nullptr;      // workspace: kBatchMaxIters * kBatchPhases * G segments
    int* hcancel = nullptr;         // pinned host word the launch's waits poll (tcol_cancel)
    int* dcancel = nullptr;         // its device view
    int* habort = nullptr;          // pinned host copy of the abort flag after a run
    int spin_limit = kBatchSpinDefault;
    int cus = 0;
    size_t ps_lds = 0;              // dynamic LDS of the sparse penalty kernel
    size_t prep_lds = 0;            // dynamic LDS of the class-size kernel
    int total_ps = 0;               // blocks of the sparse penalty kernel (0: no graph uses it)
    int total_rows = 0, total_mem = 0, total_mt = 0, total_ex = 0;
    int total_gm[2] = {0, 0};
    int kmax = 0, nmax = 0;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};   // [0] = unroll steps, [1] = one step
    hipGraph_t graph[2] = {nullptr, nullptr};
    int graph_unroll = 0;
    int graph_fused = -1;
};

#define HIPCHK(x)                                                                   \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess) {                                                     \
            fprintf(stderr, "libtcol: %s failed: %s\n", #x, hipGetErrorString(e_)); \
            return TCOL_EHIP;                                                       \
        }                                                                           \
    } while (0)

#define HIPRET(x)                                   \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return e_;            \
    } while (0)

static void drop_graphs(tcol_ctx* c) {
    for (int i = 0; i < 2; ++i) {
        if (c->gexec[i]) hipGraphExecDestroy(c->gexec[i]);
        if (c->graph[i]) hipGraphDestroy(c->graph[i]);
        c->gexec[i] = nullptr;
        c->graph[i] = nullptr;
    }
    c->graph_unroll = 0;
    c->graph_fused = -1;
}

static int common_precision(const tcol_ctx* c) {
    int prec = c->params[0].precision;
    for (auto& p : c->params)
        if (p.precision != prec) return -1;
    return prec;
}

static bool shape_listed(int bm, int ntw) {
    for (auto& s : kShapes)
        if (s[0] == bm && s[1] == ntw) return true;
    return false;
}

// tiles of a shape over all graphs
static long long tiles_for(const tcol_ctx* c, int bm, int ntw, int mode) {
    long long t = 0;
    const int BN = gemm_bn(ntw);
    for (int g = 0; g < c->G; ++g) {
        const auto& p = c->params[g];
        const int tm = c->layouts[g].n_pad / bm;
        int tn;
        if (mode == 1) {
            if (BN < p.k) return -1;
            tn = ceil_div(p.D, BN / p.k);
        } else {
            tn = ceil_div(p.D * p.k, BN);
        }
        t += (long long)tm * tn;
    }
    return t;
}

// Estimated time of one contraction launch with a tile shape: tiles run in
// rounds of (CUs x resident blocks), and a tile costs its MFMA work (BM x BN per
// K-stage) plus its operand staging (BM + BN rows per K-stage).
static double shape_cost(const tcol_ctx* c, int bm, int ntw) {
    const long long tiles = tiles_for(c, bm, ntw, 0);
    const int bn = gemm_bn(ntw);
    // 256-row tiles run one 8-wave block per CU; the others keep three stage buffers, or
    // two when only two fit two 4-wave blocks per CU
    const int waves = bm == 256 ? 8 : 4;
    const int stage = (bm + bn) * 128;
    const int per_cu = waves == 8 ? 1 : ((3 * stage <= 80 * 1024 || 2 * stage <= 80 * 1024) ? 2 : 1);
    const long long rounds = (tiles + 256LL * per_cu - 1) / (256LL * per_cu);
    // an 8-wave block measured slower than two independent 4-wave blocks of half its
    // size (their barriers do not align), so it gets no credit for its extra waves
    return (double)rounds * ((double)bm * bn + 32.0 * (bm + bn));
}

// tile shapes: options first, else the listed shape of least estimated time
static void pick_shapes(tcol_ctx* c) {
    const int prec = std::max(0, common_precision(c));
    GemmShape s{prec, 128, 8, 0};
    double best = -1.0;
    for (auto& sh : kShapes) {
        const double cost = shape_cost(c, sh[0], sh[1]);
        // ties go to the larger tile (fewer operand re-reads)
        if (best < 0.0 || cost < best || (cost == best && sh[0] * sh[1] > s.bm * s.ntw)) {
            best = cost;
            s.bm = sh[0];
            s.ntw = sh[1];
        }
    }
    if (c->opt.tile_bm && c->opt.tile_ntw && shape_listed(c->opt.tile_bm, c->opt.tile_ntw)) {
        s.bm = c->opt.tile_bm;
        s.ntw = c->opt.tile_ntw;
    }
    // the batch launch runs its own contraction tile
    if (c->opt.fused == 3) {
        s.bm = kBatchBM;
        s.ntw = kBatchNTW;
    }
    c->shape = s;
    // fused: whole members per column tile, so 32 * ntw >= k; the smallest such width,
    // with 128-row blocks when that still gives at least 512 tiles
    GemmShape f{prec, 0, 0, 1};
    if (c->opt.tile_bm && c->opt.tile_ntw && shape_listed(c->opt.tile_bm, c->opt.tile_ntw) &&
        tiles_for(c, c->opt.tile_bm, c->opt.tile_ntw, 1) > 0) {
        f.bm = c->opt.tile_bm;
        f.ntw = c->opt.tile_ntw;
    } else {
        for (int ntw : {2, 4, 8, 9}) {
            if (gemm_bn(ntw) < c->kmax) continue;
            f.ntw = ntw;
            f.bm = shape_listed(64, ntw) ? 64 : 128;
            if (shape_listed(128, ntw) && tiles_for(c, 128, ntw, 1) >= 512) f.bm = 128;
            break;
        }
    }
    c->fshape = f;
    c->fused_ok = f.ntw > 0 && common_precision(c) >= 0;
}

// Automatic penalty mode.  A balanced colouring gives each row about D n / k class-mates,
// and the per-iteration choice takes the sparse rows only while the rows average at most
// n of them: graphs with 4 D > k start too close to that bound (and from k < D above it), so
// they keep the dense operand pass (and skip the class lists).  Otherwise the choice is made per iteration, and
// partitioning, whose rows are dense either way, always takes the sparse rows.  Below a
// floor on n the dense pass is the faster route anyway: on G(n, .5) with k = n / 14.3
// the two cost the same at n = 2600-2900 for colouring (D = 16 and 32, fp4 and bf16
// operands; the dense pass 2-22 % faster below) and at about n = 2000 for partitioning
// (D = 32, fp4; 15 % faster at n = 1000).  Penalty 3 drops the floors.
constexpr int kSparseMinN = 2750, kSparseMinNPartition = 2048;
static bool sparse_preferred(const tcol_graph_params& p, bool size_floor) {
    if (p.problem == TCOL_MCOL) return false;
    if (p.problem == TCOL_KPART || p.problem == TCOL_BKPART) return !size_floor || p.n >= kSparseMinNPartition;
    return 4LL * p.D <= p.k && (!size_floor || p.n >= kSparseMinN);
}

// Members per accumulator group PM of the sparse penalty kernel: 8 (a list entry's colours in
// the group are one 16-byte word of the vertex-major colours), and the block size whose LDS
// keeps the most blocks per CU: four 512-thread blocks (40 KB), else three (53 KB), two
// (80 KB), else one of 1024 threads (160 KB).  Rows in flight count for more than fewer member
// groups per row.  Returns false when the group's LDS does not fit.
static bool pick_sparse(int kmax, int dmax, int nmax, int& PM, int& threads) {
    for (size_t budget : {(size_t)40 * 1024, (size_t)53 * 1024, (size_t)80 * 1024, (size_t)160 * 1024})
        if (penalty_sparse_lds(8, kmax, dmax, nmax) <= budget) {
            PM = 8;
            threads = budget > 80 * 1024 ? 1024 : 512;
            return true;
        }
    return false;
}

static int path_of(const tcol_ctx* c);

// The batch launch (fused = 3): whether it can run these graphs, and its item segments.  It
// runs the fast schedule with the dense penalty pass, so no graph may take the sparse rows,
// heavy-ball steps or multiple colours, and the graphs share one operand precision.  Items
// per graph and phase: class sizes (D) + expansion (groups of kBatchExpand blocks); group
// concentration (groups of kBatchMtilde tiles); contraction tiles; fitness (1); row update
// (groups of kBatchRowGroups x 16 rows).  Segments go by iteration, phase, then graph in
// decreasing tile cost (`order`); a segment's items wait for all earlier items of its graph.
static tcol_status build_batch(tcol_ctx* c, const std::vector<int>& order) {
    c->batch_ok = false;
    if (c->opt.fused != 3) return TCOL_OK;
    const int prec = common_precision(c);
    const int kpl = batch_kpl(c->kmax);
    if (c->total_ps > 0 || c->any_momentum || c->any_mcol || prec < 0 || kpl == 0 || !update_rows_kpl(c->kmax))
        return TCOL_OK;
    const int G = c->G;
    std::vector<std::array<int, kBatchPhases>> items(G);
    long long per_iter = 0;
    for (int g = 0; g < G; ++g) {
        const GraphDev& d = c->hdesc[g];
        const auto& p = c->params[g];
        items[g][0] = p.D + ceil_div(d.ex_cblocks, kBatchExpand);
        items[g][1] = ceil_div(c->layouts[g].mt_tiles, kBatchMtilde);
        items[g][2] = d.gm_tm[0] * d.gm_tn[0];
        items[g][3] = 1;
        items[g][4] = ceil_div(p.D * p.n, 16 * kBatchRowGroups);
        for (int ph = 0; ph < kBatchPhases; ++ph) per_iter += items[g][ph];
    }
    if (per_iter * kBatchMaxIters >= (1LL << 30)) return TCOL_OK;
    std::vector<BatchSeg> segs;
    segs.reserve((size_t)kBatchMaxIters * kBatchPhases * G);
    int start = 0;
    for (int it = 0; it < kBatchMaxIters; ++it)
        for (int ph = 0; ph < kBatchPhases; ++ph)
            for (int g : order) {
                int before = 0;
                for (int q = 0; q < kBatchPhases; ++q) before += items[g][q];
                int need = it * before;
                for (int q = 0; q < ph; ++q) need += items[g][q];
                BatchSeg sg{};
                sg.start = start;
                sg.g = g;
                sg.phase = ph;
                sg.iter = it;
                sg.need = need;
                segs.push_back(sg);
                start += items[g][ph];
            }
    int bpc = 0;
    HIPCHK(batch_prepare(prec, kpl, &bpc));
    if (bpc < 1) return TCOL_OK;
    HIPCHK(hipMemcpyAsync(c->dsegs, segs.data(), sizeof(BatchSeg) * segs.size(), hipMemcpyHostToDevice, c->stream));
    c->batch_prec = prec;
    c->batch_kpl = kpl;
    c->batch_items = (int)per_iter;
    c->batch_lds = batch_lds_bytes(prec, c->prep_lds);
    c->batch_ok = true;
    return TCOL_OK;
}

// recompute flattened work offsets for the tile shapes and upload the descriptors
static tcol_status rebuild_schedule(tcol_ctx* c) {
    pick_shapes(c);
    HIPCHK(gemm_prepare(c->shape));
    if (c->fused_ok) HIPCHK(gemm_prepare(c->fshape));
    HIPCHK(penalty_sparse_prepare());
    const int BN0 = gemm_bn(c->shape.ntw);
    const int BN1 = c->fused_ok ? gemm_bn(c->fshape.ntw) : 0;
    // sparse penalty: a graph takes it on request (penalty 2) or when the automatic choice
    // prefers it
    int ps_k = 0, ps_D = 0, ps_n = 0;
    for (int g = 0; g < c->G; ++g) {
        const tcol_graph_params& p = c->params[g];
        const int pen = c->opt.penalty;
        c->hdesc[g].psparse =
            p.problem != TCOL_MCOL && (pen == 2 || ((pen == 0 || pen == 3) && sparse_preferred(p, pen == 0))) ? 1 : 0;
        c->hdesc[g].ps_mode = pen == 2 ? 1 : 2;
        if (c->hdesc[g].psparse) {
            ps_k = std::max(ps_k, p.k);
            ps_D = std::max(ps_D, p.D);
            ps_n = std::max(ps_n, p.n);
        }
    }
    c->ps_PM = c->ps_threads = c->ps_kw = 0;
    c->ps_lds = 0;
    for (int g = 0; g < c->G; ++g) c->hdesc[g].pfuse = 0;
    if (ps_k > 0) {
        // graphs too large for the kernel's LDS take the dense pass
        int PM = 0, threads = 0;
        if (pick_sparse(ps_k, ps_D, ps_n, PM, threads)) {
            // on the fast path the sparse rows also take the row update of their graphs (one
            // wave per member of a group, so at most threads / 64 members per group), in every
            // iteration, unless a graph takes heavy-ball steps (its velocity is updated in place,
            // which an update discarded by the stop rule could not undo)
            const int kw = penalty_sparse_kw(ps_k);
            if (path_of(c) == 1 && kw > 0) {
                for (int g = 0; g < c->G; ++g)
                    if (c->hdesc[g].psparse && c->params[g].momentum == 0.0f) c->hdesc[g].pfuse = 1;
                c->ps_kw = kw;
                PM = std::min(PM, threads / 64 / 8 * 8);
            }
            c->ps_PM = PM;
            c->ps_threads = threads;
            c->ps_lds = penalty_sparse_lds(PM, ps_k, ps_D, ps_n);
        } else {
            for (int g = 0; g < c->G; ++g) c->hdesc[g].psparse = 0;
            ps_k = 0;
        }
    }
    c->all_pfuse = true;
    for (int g = 0; g < c->G; ++g)
        if (!c->hdesc[g].pfuse) c->all_pfuse = false;
    c->prep_lds = prep_lds(c->kmax, c->nmax, ps_k > 0);
    int rows = 0, mem = 0, pg = 0, mt = 0, ex = 0;
    for (int g = 0; g < c->G; ++g) {
        const tcol_graph_params& p = c->params[g];
        const Layout& L = c->layouts[g];
        GraphDev& d = c->hdesc[g];
        d.row_begin = rows;
        rows += p.D * p.n;
        d.mem_begin = mem;
        mem += p.D;
        d.ps_begin = pg;
        if (d.psparse) pg += p.n;
        d.mt_begin = mt;
        d.mt_T = L.mt_T;
        d.mt_ts = L.mt_ts;
        mt += L.mt_tiles;
        d.ex_begin = ex;
        d.ex_cblocks = expand_blocks(p.D, p.k, L.n_pad);
        ex += d.ex_cblocks;
        d.gm_tm[0] = L.n_pad / c->shape.bm;
        d.gm_tn[0] = ceil_div(p.D * p.k, BN0);
        if (c->fused_ok) {
            d.gm_mpb = BN1 / p.k;
            d.gm_tm[1] = L.n_pad / c->fshape.bm;
            d.gm_tn[1] = ceil_div(p.D, d.gm_mpb);
        }
    }
    // contraction tiles: the graphs' ranges in decreasing K (= n_pad, the length of a tile's
    // sweep), so a batch's longest tiles start first and short ones fill the end
    std::vector<int> order(c->G);
    for (int g = 0; g < c->G; ++g) order[g] = g;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return c->layouts[a].n_pad > c->layouts[b].n_pad; });
    int gm0 = 0, gm1 = 0;
    for (int g : order) {
        GraphDev& d = c->hdesc[g];
        d.gm_begin[0] = gm0;
        gm0 += d.gm_tm[0] * d.gm_tn[0];
        if (c->fused_ok) {
            d.gm_begin[1] = gm1;
            gm1 += d.gm_tm[1] * d.gm_tn[1];
        }
    }
    c->total_rows = rows;
    c->total_mem = mem;
    c->total_ps = pg;
    c->total_mt = mt;
    c->total_ex = ex;
    c->total_gm[0] = gm0;
    c->total_gm[1] = gm1;
    tcol_status bs = build_batch(c, order);
    if (bs != TCOL_OK) return bs;
    HIPCHK(hipMemcpyAsync(c->ddesc, c->hdesc.data(), sizeof(GraphDev) * c->G, hipMemcpyHostToDevice, c->stream));
    drop_graphs(c);
    return TCOL_OK;
}

// step schedule actually used: 2 needs the epilogue tiling, 1 needs the row-update kernel
static int path_of(const tcol_ctx* c) {
    if (c->any_mcol) return 0;
    if (c->opt.fused == 3 && c->batch_ok) return 3;
    if (c->opt.fused == 2 && c->fused_ok && !c->any_momentum) return 2;
    if (c->opt.fused >= 1 && update_rows_kpl(c->kmax)) return 1;
    return 0;
}
static bool use_fused(const tcol_ctx* c) { return path_of(c) == 2; }

static hipError_t launch_update_any(tcol_ctx* c, int honor, int mode, int gsel, float* gs, float* gw, hipStream_t s) {
    if (update_rows_kpl(c->kmax))
        return launch_update_rows(c->ddesc, c->G, c->total_rows, c->kmax, c->update_var, honor, mode, gsel, gs, gw, s);
    return launch_update(c->ddesc, c->G, c->total_rows, honor, mode, gsel, gs, gw, s);
}

// ---------------------------------------------------------------- sequences --

// one Algorithm-1 iteration for every running graph (plain path)
static hipError_t enqueue_step_plain(tcol_ctx* c, hipStream_t s) {
    HIPRET(launch_colors(c->ddesc, c->G, c->total_rows, 1, s));
    HIPRET(launch_prep(c->ddesc, c->G, c->total_mem, c->prep_lds, 1, 0, 0, 0, 0, s));
    HIPRET(launch_expand(c->ddesc, c->G, c->total_ex, 1, 0, 0, s));
    HIPRET(launch_mtilde(c->ddesc, c->G, c->total_mt, 1, 0, -1, nullptr, s));
    HIPRET(launch_gemm(c->shape, c->ddesc, c->G, c->total_gm[0], 1, 15, 0, s));
    HIPRET(launch_fitness(c->ddesc, c->G, 1, kFlagPlainPen, -1, s));
    HIPRET(launch_update_any(c, 1, 0, -1, nullptr, nullptr, s));
    HIPRET(launch_advance(c->ddesc, c->G, s));
    return hipSuccess;
}

// penalty of the fast and epilogue paths: sparse penalty rows or the dense operand, per
// graph and, for graphs that choose per iteration, per iteration (by launch_prep).  On
// the epilogue path the sparse rows go to G before the contraction, whose epilogue adds
// them; the fast path adds them to the contraction's G afterwards (enqueue_sparse_add).
static hipError_t enqueue_penalty(tcol_ctx* c, hipStream_t s) {
    if (c->total_ps > 0 && path_of(c) == 2)
        HIPRET(launch_penalty_sparse(c->ddesc, c->G, c->total_ps, c->ps_PM, c->ps_threads, 0, 0, c->ps_lds, 1, 0, s));
    HIPRET(launch_mtilde(c->ddesc, c->G, c->total_mt, 1, kFlagGate, -1, nullptr, s));
    return hipSuccess;
}

// class sizes and lists of the current colours, then (fast and epilogue paths) the
// iteration's penalty choice, which the expansion, penalty and contraction read
static hipError_t enqueue_prep(tcol_ctx* c, hipStream_t s) {
    HIPRET(launch_prep(c->ddesc, c->G, c->total_mem, c->prep_lds, 1, 0, c->total_ps > 0 ? 1 : 0, 0, 0, s));
    return hipSuccess;
}

// fast path: the sparse rows added to the contraction's G (they also gather f_color for the
// graphs that take them, into slots the fitness folds), and for graphs with pfuse the row
// update, in every iteration, into the other W and colour buffers; with `fitness` the fitness
// launch follows (which accepts those updates unless the graph stops), else the caller
// launches it
static hipError_t enqueue_sparse_add(tcol_ctx* c, bool fitness, hipStream_t s) {
    if (c->total_ps > 0)
        HIPRET(launch_penalty_sparse(c->ddesc, c->G, c->total_ps, c->ps_PM, c->ps_threads, c->ps_kw,
                                     c->update_var & 1, c->ps_lds, 1, 1, s));
    if (fitness) HIPRET(launch_fitness(c->ddesc, c->G, 1, kFlagFoldSparse | kFlagFlipFused, -1, s));
    return hipSuccess;
}

// whether some graph computes A.S in fp8: its expansion writes the bf16 copy of S only in
// the iterations that take the dense pass, so it has to follow the penalty choice
static bool any_split(const tcol_ctx* c) {
    for (int g = 0; g < c->G; ++g)
        if (prec_split(c->params[g].precision)) return true;
    return false;
}

// one iteration on the fast path; c[pS] holds the colours of the current weights.  The
// expansion reads only the colours, so unless it depends on the penalty choice its
// blocks ride on the class-size launch
// blocks ride on the class-size launch.  In a run of iterations the class-size launch
// also ends the previous one (advance_prev), and only the last iteration launches its own
// end (advance_own)
static hipError_t enqueue_step_fast(tcol_ctx* c, bool advance_prev, bool advance_own, hipStream_t s) {
    const bool merged = !any_split(c);
    HIPRET(launch_prep(c->ddesc, c->G, c->total_mem, c->prep_lds, 1, 0, c->total_ps > 0 ? 1 : 0,
                       merged ? c->total_ex : 0, advance_prev ? 1 : 0, s));
    HIPRET(enqueue_penalty(c, s));
    if (!merged) HIPRET(launch_expand(c->ddesc, c->G, c->total_ex, 1, 0, 1, s));
    HIPRET(launch_gemm(c->shape, c->ddesc, c->G, c->total_gm[0], 1, 7 | 32 | 64, 0, s));
    HIPRET(enqueue_sparse_add(c, true, s));
    // the row update of the graphs whose update did not ride on the sparse rows
    if (!c->all_pfuse)
        HIPRET(launch_update_rows(c->ddesc, c->G, c->total_rows, c->kmax, c->update_var, 1, 0, -1, nullptr, nullptr, s));
    if (advance_own) HIPRET(launch_advance(c->ddesc, c->G, s));
    return hipSuccess;
}

// one iteration on the epilogue path; c[pS] holds the colours of the current weights
static hipError_t enqueue_step_fused(tcol_ctx* c, hipStream_t s) {
    HIPRET(enqueue_prep(c, s));
    HIPRET(enqueue_penalty(c, s));
    HIPRET(launch_expand(c->ddesc, c->G, c->total_ex, 1, 0, 1, s));
    HIPRET(launch_gemm(c->fshape, c->ddesc, c->G, c->total_gm[1], 1, 7, 0, s));
    HIPRET(launch_fitness(c->ddesc, c->G, 1, kFlagFused, -1, s));
    return hipSuccess;
}

// runs of up to kBatchMaxIters iterations, each one batch launch (the counters cleared by a
// fill kernel first) and the run's last counter advance
static hipError_t enqueue_batch(tcol_ctx* c, int n, hipStream_t s) {
    const size_t ctl = batch_ctl_bytes(c->G);
    for (int done = 0; done < n;) {
        const int run = std::min(kBatchMaxIters, n - done);
        HIPRET(launch_zero(c->dctl + 4, ctl - 4 * sizeof(int), s));
        const int total = run * c->batch_items;
        HIPRET(launch_batch_run(c->batch_prec, c->batch_kpl, total, c->batch_lds, c->ddesc, c->G, c->dsegs,
                                run * kBatchPhases * c->G, total, c->dctl, c->dcancel, c->spin_limit, s));
        HIPRET(launch_advance(c->ddesc, c->G, s));
        done += run;
    }
    return hipSuccess;
}

static hipError_t enqueue_steps(tcol_ctx* c, int n, hipStream_t s) {
    const int path = path_of(c);
    if (path == 3) return enqueue_batch(c, n, s);
    for (int i = 0; i < n; ++i)
        HIPRET(path == 2 ? enqueue_step_fused(c, s)
                         : (path == 1 ? enqueue_step_fast(c, i > 0, i == n - 1, s) : enqueue_step_plain(c, s)));
    return hipSuccess;
}

static tcol_status build_graphs(tcol_ctx* c) {
    drop_graphs(c);
    const int U = std::max(1, std::min(64, c->opt.unroll));
    const int counts[2] = {U, 1};
    for (int i = 0; i < 2; ++i) {
        HIPCHK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_steps(c, counts[i], c->cap);
        hipGraph_t gr = nullptr;
        hipError_t e2 = hipStreamEndCapture(c->cap, &gr);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (gr) hipGraphDestroy(gr);
            fprintf(stderr, "libtcol: graph capture failed: %s\n", hipGetErrorString(e != hipSuccess ? e : e2));
            return TCOL_EHIP;
        }
        c->graph[i] = gr;
        HIPCHK(hipGraphInstantiate(&c->gexec[i], gr, nullptr, nullptr, 0));
    }
    c->graph_unroll = U;
    c->graph_fused = path_of(c);
    return TCOL_OK;
}

// run `steps` iterations (graph replays or eager launches); no synchronisation
static tcol_status run_steps(tcol_ctx* c, int steps) {
    if (steps <= 0) return TCOL_OK;
    // the batch launch's abort flag holds for the whole call
    if (path_of(c) == 3) HIPCHK(launch_zero(c->dctl, 4 * sizeof(int), c->stream));
    // the fast and epilogue paths colour the updated rows themselves: one argmax pass first
    if (path_of(c) != 0) HIPCHK(launch_colors(c->ddesc, c->G, c->total_rows, 1, c->stream));
    if (c->opt.use_graph) {
        const int U = std::max(1, std::min(64, c->opt.unroll));
        if (c->graph_unroll != U || !c->gexec[0] || c->graph_fused != path_of(c)) {
            tcol_status s = build_graphs(c);
            if (s != TCOL_OK) return s;
        }
        for (int i = 0; i < steps / U; ++i) HIPCHK(hipGraphLaunch(c->gexec[0], c->stream));
        for (int i = 0; i < steps % U; ++i) HIPCHK(hipGraphLaunch(c->gexec[1], c->stream));
    } else {
        HIPCHK(enqueue_steps(c, steps, c->stream));
    }
    return TCOL_OK;
}

// read the graph states (synchronises) and move fused-path weights back into the caller's buffer
static tcol_status settle(tcol_ctx* c) {
    HIPCHK(hipMemcpyAsync(c->hstate, c->dstate, sizeof(GraphState) * c->G, hipMemcpyDeviceToHost, c->stream));
    if (c->batch_ok) HIPCHK(hipMemcpyAsync(c->habort, c->dctl, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    bool any = false;
    for (int g = 0; g < c->G; ++g) {
        if (c->hstate[g].pW == 1) {
            const auto& p = c->params[g];
            HIPCHK(hipMemcpyAsync(c->hdesc[g].W[0], c->hdesc[g].W[1], sizeof(float) * (size_t)p.D * p.n * p.k,
                                  hipMemcpyDeviceToDevice, c->stream));
            any = true;
        }
    }
    if (any) HIPCHK(launch_state(c->ddesc, c->G, 3, -1, 0, c->stream));
    // a wait of the batch launch gave up (the host's cancel word or the wait limit)
    if (c->batch_ok && c->habort[0]) {
        // the run stopped part-way: clear the flag and the conflict accumulators the
        // contraction tiles of unfinished iterations left behind
        c->habort[0] = 0;
        HIPCHK(launch_zero(c->dctl, 4 * sizeof(int), c->stream));
        HIPCHK(launch_state(c->ddesc, c->G, 4, -1, 0, c->stream));
        return TCOL_EABORT;
    }
    return TCOL_OK;
}

// ---------------------------------------------------------------- C ABI ------

extern "C" {

const char* tcol_status_string(tcol_status s) {
    switch (s) {
        case TCOL_OK: return "ok";
        case TCOL_EINVAL: return "invalid argument";
        case TCOL_ESHAPE: return "unsupported shape";
        case TCOL_EGRAPH: return "adjacency matrix is not symmetric 0/1 with a zero diagonal";
        case TCOL_EHIP: return "HIP runtime error";
        case TCOL_ENONFINITE: return "non-finite weight";
        case TCOL_ENOMEM: return "out of device memory or workspace too small";
        case TCOL_ESTATE: return "invalid state";
        case TCOL_EABORT: return "a wait of the batch launch gave up (cancelled, or past the wait limit)";
        default: return "unknown status";
    }
}

tcol_status tcol_workspace_size(int32_t G, const tcol_graph_params* p, size_t* bytes) {
    if (G < 1 || !p || !bytes) return TCOL_EINVAL;
    size_t tot = head_bytes(G);
    for (int g = 0; g < G; ++g) {
        tcol_status s = check_params(p[g]);
        if (s != TCOL_OK) return s;
        tot += make_layout(p[g]).total;
    }
    *bytes = tot;
    return TCOL_OK;
}

void tcol_destroy(tcol_ctx* c) {
    if (!c) return;
    if (c->stream) hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->cap) hipStreamDestroy(c->cap);
    if (c->ws_owned && c->ws) hipFree(c->ws);
    if (c->hstate) hipHostFree(c->hstate);
    if (c->hcancel) hipHostFree(c->hcancel);
    delete c;
}

// report a failed HIP step of tcol_init with the runtime's last error
static tcol_status init_fail(const char* what) {
    fprintf(stderr, "libtcol: init: %s failed: %s\n", what, hipGetErrorString(hipGetLastError()));
    return TCOL_EHIP;
}

tcol_status tcol_init(tcol_ctx** out, int32_t G, const tcol_graph_params* p, const uint8_t* const* A_dev,
                      float* const* W_dev, void* ws_dev, size_t ws_bytes, void* stream) {
    if (!out) return TCOL_EINVAL;
    *out = nullptr;
    if (G < 1 || !p || !A_dev || !W_dev) return TCOL_EINVAL;
    size_t need = 0;
    tcol_status s = tcol_workspace_size(G, p, &need);
    if (s != TCOL_OK) return s;
    for (int g = 0; g < G; ++g)
        if (!A_dev[g] || !W_dev[g]) return TCOL_EINVAL;
    if (ws_dev && ws_bytes < need) return TCOL_ENOMEM;

    tcol_ctx* c = new tcol_ctx();
    c->G = G;
    c->stream = (hipStream_t)stream;
    c->params.assign(p, p + G);
    c->opt.fused = 1;
    c->opt.use_graph = 1;
    c->opt.unroll = 8;
    for (auto& q : c->params) {
        c->kmax = std::max(c->kmax, q.k);
        c->nmax = std::max(c->nmax, q.n);
        if (q.momentum != 0.0f) c->any_momentum = true;
        if (q.momentum != 0.0f) c->update_var |= 2;
        if (q.problem == TCOL_MCOL) c->any_mcol = true;
        if (prob_added(q.problem) && q.nu != 0.0f) c->update_var |= 1;
    }
    if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
        fprintf(stderr, "libtcol: capture stream creation failed\n");
        delete c;
        return TCOL_EHIP;
    }
    if (hipHostMalloc((void**)&c->hstate, sizeof(GraphState) * G, hipHostMallocDefault) != hipSuccess) {
        tcol_destroy(c);
        return TCOL_ENOMEM;
    }
    // the batch launch's cancel word (polled by its waits) and the abort flag's host copy
    if (hipHostMalloc((void**)&c->hcancel, 64, hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer((void**)&c->dcancel, c->hcancel, 0) != hipSuccess) {
        tcol_destroy(c);
        return TCOL_ENOMEM;
    }
    c->hcancel[0] = 0;
    c->habort = c->hcancel + 4;
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            tcol_destroy(c);
            return TCOL_EHIP;
        }
    }
    if (ws_dev) {
        c->ws = (uint8_t*)ws_dev;
        c->ws_bytes = ws_bytes;
    } else {
        if (hipMalloc((void**)&c->ws, need) != hipSuccess) {
            c->ws = nullptr;
            tcol_destroy(c);
            return TCOL_ENOMEM;
        }
        c->ws_owned = true;
        c->ws_bytes = need;
    }
    // every buffer starts at zero: padding rows/columns of the operands stay zero forever
    if (hipMemsetAsync(c->ws, 0, need, c->stream) != hipSuccess) {
        fprintf(stderr, "libtcol: clearing the workspace (%zu bytes) failed\n", need);
        tcol_destroy(c);
        return TCOL_EHIP;
    }
    c->ddesc = (GraphDev*)c->ws;
    c->dstate = (GraphState*)(c->ws + align_up(sizeof(GraphDev) * G));
    c->dctl = (int*)(c->ws + align_up(sizeof(GraphDev) * G) + align_up(sizeof(GraphState) * G));
    c->dsegs = (BatchSeg*)((uint8_t*)c->dctl + batch_ctl_bytes(G));
    size_t off = head_bytes(G);
    c->hdesc.resize(G);
    c->layouts.resize(G);
    // graph check flag, then (8-byte aligned) one count of A's ones per graph
    int* dbad = nullptr;
    const size_t chk_bytes = 8 + sizeof(unsigned long long) * G;
    if (hipMalloc((void**)&dbad, chk_bytes) != hipSuccess ||
        hipMemsetAsync(dbad, 0, chk_bytes, c->stream) != hipSuccess) {
        fprintf(stderr, "libtcol: graph check flag allocation failed\n");
        if (dbad) hipFree(dbad);
        tcol_destroy(c);
        return TCOL_EHIP;
    }
    tcol_status rc = TCOL_OK;
    for (int g = 0; g < G && rc == TCOL_OK; ++g) {
        const tcol_graph_params& q = p[g];
        Layout L = make_layout(q);
        c->layouts[g] = L;
        uint8_t* b = c->ws + off;
        off += L.total;
        GraphDev& d = c->hdesc[g];
        memset(&d, 0, sizeof(d));
        d.n = q.n;
        d.k = q.k;
        d.D = q.D;
        d.n_pad = L.n_pad;
        d.cs = round_up(q.n, 64);
        d.ncols = q.D * q.k;
        d.rows_S = L.rows_S;
        d.problem = q.problem;
        d.precision = q.precision;
        d.bonus_diag = q.bonus_diag ? 1 : 0;
        d.stop_on_legal = q.stop_on_legal ? 1 : 0;
        d.nb_iter = q.nb_iter;
        d.c1 = q.n / q.k;
        d.c2 = (q.n % q.k == 0) ? q.n / q.k : q.n / q.k + 1;
        d.eta = q.eta;
        d.rho = q.rho;
        d.nu = prob_added(q.problem) ? q.nu : 0.0f;
        d.momentum = q.momentum;
        d.vel = q.momentum != 0.0f ? (float*)(b + L.off[B_VEL]) : nullptr;
        d.lambda = q.lambda;
        d.mu = q.mu;
        d.lut_pen = (const float*)(b + L.off[B_LUT_PEN]);
        d.lut_bon = (const float*)(b + L.off[B_LUT_BON]);
        d.lut_ka = (const double*)(b + L.off[B_LUT_KA]);
        d.lut_vb = (const double*)(b + L.off[B_LUT_VB]);
        d.W[0] = W_dev[g];
        d.W[1] = (float*)(b + L.off[B_W2]);
        d.A8 = b + L.off[B_A8];
        d.Aop = b + L.off[B_AOP];
        d.Pop = b + L.off[B_POP];
        d.Sop[0] = b + L.off[B_S0];
        d.Sop[1] = b + L.off[B_S1];
        d.Sp2[0] = prec_split(q.precision) ? (void*)(b + L.off[B_SP0]) : nullptr;
        d.Sp2[1] = prec_split(q.precision) ? (void*)(b + L.off[B_SP1]) : nullptr;
        d.c[0] = (int16_t*)(b + L.off[B_C0]);
        d.c[1] = (int16_t*)(b + L.off[B_C1]);
        d.V[0] = (int32_t*)(b + L.off[B_V0]);
        d.V[1] = (int32_t*)(b + L.off[B_V1]);
        d.G = (float*)(b + L.off[B_G]);
        d.f2 = (int32_t*)(b + L.off[B_F2]);
        d.f2p = (int32_t*)(b + L.off[B_F2P]);
        d.fcol = (int64_t*)(b + L.off[B_FCOL]);
        d.feq = (int64_t*)(b + L.off[B_FEQ]);
        d.f = (int64_t*)(b + L.off[B_F]);
        d.part = (double*)(b + L.off[B_PART]);
        d.snap = (int16_t*)(b + L.off[B_SNAP]);
        d.st = c->dstate + g;
        d.cT = (int16_t*)(b + L.off[B_CT]);
        d.cTs = round_up(q.D, 8);
        d.cmax = cmax_of(q);
        d.dem = (const int32_t*)(b + L.off[B_DEM]);
        d.sel = d.cmax > 1 ? (int16_t*)(b + L.off[B_SEL]) : nullptr;
        d.cls_v = (int16_t*)(b + L.off[B_CLSV]);
        d.cls_off = (int32_t*)(b + L.off[B_CLSOFF]);
        d.cinfo = (int2*)(b + L.off[B_CINFO]);
        d.sq = (long long*)(b + L.off[B_SQ]);
        // look-up tables over the group concentration m = 0..D (host libm, FP64); for
        // partitioning the powers are of D - m (M replaced by J - M)
        const int nlut = q.D * d.cmax + 1;
        std::vector<float> lp(nlut), lb(nlut);
        std::vector<double> lka(nlut), lvb(nlut);
        for (int m = 0; m < nlut; ++m) {
            const double x = prob_partition(q.problem) ? (double)(q.D - m) : (double)m;
            lp[m] = (float)(2.0 * q.alpha * q.lambda * pow0(x, (double)q.alpha - 1.0));
            lb[m] = (float)(2.0 * q.beta * q.mu * pow0(x, (double)q.beta - 1.0));
            lka[m] = pow0(x, q.alpha);
            lvb[m] = pow0(x, q.beta);
        }
        if (hipMemcpy(b + L.off[B_LUT_PEN], lp.data(), sizeof(float) * lp.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(b + L.off[B_LUT_BON], lb.data(), sizeof(float) * lb.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(b + L.off[B_LUT_KA], lka.data(), sizeof(double) * lka.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(b + L.off[B_LUT_VB], lvb.data(), sizeof(double) * lvb.size(), hipMemcpyHostToDevice) != hipSuccess)
            rc = init_fail("look-up table upload");
        if (rc == TCOL_OK) {
            // every demand 1 until tcol_set_demand
            std::vector<int32_t> one(q.n, 1);
            if (hipMemcpy(b + L.off[B_DEM], one.data(), sizeof(int32_t) * q.n, hipMemcpyHostToDevice) != hipSuccess)
                rc = init_fail("demand upload");
        }
        if (rc == TCOL_OK &&
            launch_pack_graph(A_dev[g], q.n, L.n_pad, q.precision, (uint8_t*)d.A8, d.Aop, dbad,
                              (unsigned long long*)(dbad + 2) + g, c->stream) != hipSuccess)
            rc = init_fail("graph packing launch");
    }
    int bad = 0;
    std::vector<unsigned long long> ones(G, 0);
    if (rc == TCOL_OK) {
        if (hipMemcpyAsync(&bad, dbad, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipMemcpyAsync(ones.data(), dbad + 2, sizeof(unsigned long long) * G, hipMemcpyDeviceToHost,
                           c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            rc = init_fail("graph check");
    }
    hipFree(dbad);
    // |E|: every edge is counted from both ends
    for (int g = 0; g < G && rc == TCOL_OK; ++g) c->hdesc[g].edges = (long long)(ones[g] / 2);
    if (rc == TCOL_OK && bad) rc = TCOL_EGRAPH;
    if (rc == TCOL_OK) {
        std::vector<GraphState> st(G);
        for (auto& x : st) {
            memset(&x, 0, sizeof(x));
            x.legal_d = -1;
        }
        if (hipMemcpy(c->dstate, st.data(), sizeof(GraphState) * G, hipMemcpyHostToDevice) != hipSuccess)
            rc = init_fail("state upload");
    }
    if (rc == TCOL_OK) rc = rebuild_schedule(c);
    if (rc == TCOL_OK && hipStreamSynchronize(c->stream) != hipSuccess) rc = init_fail("set-up");
    if (rc != TCOL_OK) {
        tcol_destroy(c);
        return rc;
    }
    *out = c;
    return TCOL_OK;
}

tcol_status tcol_set_options(tcol_ctx* c, const tcol_options* o) {
    if (!c || !o) return TCOL_EINVAL;
    if (o->unroll < 0 || o->unroll > 64) return TCOL_EINVAL;
    if (o->penalty < 0 || o->penalty > 3) return TCOL_EINVAL;
    if (o->fused < 0 || o->fused > 3) return TCOL_EINVAL;
    if ((o->tile_bm || o->tile_ntw) && !shape_listed(o->tile_bm, o->tile_ntw)) return TCOL_EINVAL;
    tcol_options old = c->opt;
    c->opt = *o;
    if (c->opt.unroll == 0) c->opt.unroll = 8;
    tcol_status s = rebuild_schedule(c);
    if (s != TCOL_OK) {
        c->opt = old;
        rebuild_schedule(c);
    }
    return s;
}

tcol_status tcol_get_options(tcol_ctx* c, tcol_options* o) {
    if (!c || !o) return TCOL_EINVAL;
    *o = c->opt;
    const GemmShape& s = path_of(c) == 2 ? c->fshape : c->shape;
    if (!o->tile_bm) o->tile_bm = s.bm;
    if (!o->tile_ntw) o->tile_ntw = s.ntw;
    o->fused = path_of(c);
    return TCOL_OK;
}

tcol_status tcol_step(tcol_ctx* c, int32_t max_steps, int32_t* steps_done, int32_t* legal_d,
                      int16_t* const* colors_out_dev) {
    if (!c || max_steps < 0) return TCOL_EINVAL;
    __atomic_store_n(&c->hcancel[0], 0, __ATOMIC_RELEASE);
    HIPCHK(launch_state(c->ddesc, c->G, 0, -1, 0, c->stream));
    tcol_status rs = run_steps(c, max_steps);
    if (rs != TCOL_OK) return rs;
    tcol_status s = settle(c);
    if (s != TCOL_OK) return s;
    int done = 0;
    tcol_status rc = TCOL_OK;
    for (int g = 0; g < c->G; ++g) {
        const GraphState& st = c->hstate[g];
        done = std::max(done, st.steps_done);
        if (legal_d) legal_d[g] = st.legal_d;
        if (st.error) rc = st.error;
        if (colors_out_dev && colors_out_dev[g] && st.legal_d >= 0)
            HIPCHK(hipMemcpyAsync(colors_out_dev[g], c->hdesc[g].snap,
                                  sizeof(int16_t) * c->params[g].n * c->hdesc[g].cmax, hipMemcpyDeviceToDevice,
                                  c->stream));
    }
    if (steps_done) *steps_done = done;
    return rc;
}

tcol_status tcol_conflicts(tcol_ctx* c, int32_t g, int16_t* colors_dev, int64_t* f_color_dev, int64_t* f_eq_dev) {
    if (!c || g < 0 || g >= c->G) return TCOL_EINVAL;
    // steps 1-2 for all graphs of the context (cheap), reporting only
    HIPCHK(launch_colors(c->ddesc, c->G, c->total_rows, 0, c->stream));
    HIPCHK(launch_prep(c->ddesc, c->G, c->total_mem, c->prep_lds, 0, 0, 0, 0, 0, c->stream));
    HIPCHK(launch_expand(c->ddesc, c->G, c->total_ex, 0, 0, 0, c->stream));
    HIPCHK(launch_gemm(c->shape, c->ddesc, c->G, c->total_gm[0], 0, 1, 0, c->stream));
    HIPCHK(launch_fitness(c->ddesc, c->G, 0, kFlagReport, -1, c->stream));
    HIPCHK(launch_copy_report(c->ddesc, g, colors_dev, f_color_dev, f_eq_dev, c->stream));
    return TCOL_OK;
}

tcol_status tcol_loss_grad(tcol_ctx* c, int32_t g, double* loss_dev, float* gradS_dev, float* gradW_dev) {
    if (!c || g < 0 || g >= c->G) return TCOL_EINVAL;
    HIPCHK(launch_colors(c->ddesc, c->G, c->total_rows, 0, c->stream));
    HIPCHK(launch_prep(c->ddesc, c->G, c->total_mem, c->prep_lds, 0, 0, 0, 0, 0, c->stream));
    HIPCHK(launch_expand(c->ddesc, c->G, c->total_ex, 0, 0, 0, c->stream));
    HIPCHK(launch_mtilde(c->ddesc, c->G, c->total_mt, 0, kFlagLoss | kFlagForcePen, g, nullptr, c->stream));
    HIPCHK(launch_gemm(c->shape, c->ddesc, c->G, c->total_gm[0], 0, 15, 0, c->stream));
    HIPCHK(launch_fitness(c->ddesc, c->G, 0, kFlagReport, -1, c->stream));
    if (loss_dev) HIPCHK(launch_loss(c->ddesc, g, c->layouts[g].mt_tiles, loss_dev, c->stream));
    if (gradS_dev || gradW_dev) HIPCHK(launch_update_any(c, 0, 1, g, gradS_dev, gradW_dev, c->stream));
    return TCOL_OK;
}

tcol_status tcol_class_conflicts(tcol_ctx* c, int32_t g, int32_t* C_dev) {
    if (!c || g < 0 || g >= c->G || !C_dev) return TCOL_EINVAL;
    if (c->params[g].problem == TCOL_MCOL) return TCOL_EINVAL;
    // colours and S of the current W, then A.S stored to G (no penalty pass, no gather)
    HIPCHK(launch_colors(c->ddesc, c->G, c->total_rows, 0, c->stream));
    HIPCHK(launch_prep(c->ddesc, c->G, c->total_mem, c->prep_lds, 0, 0, 0, 0, 0, c->stream));
    HIPCHK(launch_expand(c->ddesc, c->G, c->total_ex, 0, 0, 0, c->stream));
    HIPCHK(launch_gemm(c->shape, c->ddesc, c->G, c->total_gm[0], 0, 1 | 4 | 16 | 128, 0, c->stream));
    HIPCHK(launch_class_conflicts(c->ddesc, g, c->params[g].D, c->params[g].k, C_dev, c->stream));
    return TCOL_OK;
}

tcol_status tcol_set_demand(tcol_ctx* c, int32_t g, const int32_t* demand) {
    if (!c || g < 0 || g >= c->G || !demand) return TCOL_EINVAL;
    const tcol_graph_params& p = c->params[g];
    if (p.problem != TCOL_MCOL) return TCOL_EINVAL;
    for (int i = 0; i < p.n; ++i)
        if (demand[i] < 1 || demand[i] > c->hdesc[g].cmax) return TCOL_EINVAL;
    HIPCHK(hipMemcpyAsync(const_cast<int32_t*>(c->hdesc[g].dem), demand, sizeof(int32_t) * p.n, hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return TCOL_OK;
}

tcol_status tcol_selection(tcol_ctx* c, int32_t g, int16_t* sel_dev) {
    if (!c || g < 0 || g >= c->G || !sel_dev) return TCOL_EINVAL;
    HIPCHK(launch_colors(c->ddesc, c->G, c->total_rows, 0, c->stream));
    HIPCHK(launch_copy_selection(c->ddesc, g, sel_dev, c->stream));
    return TCOL_OK;
}

tcol_status tcol_mtilde(tcol_ctx* c, int32_t g, int32_t* mt_dev) {
    if (!c || g < 0 || g >= c->G || !mt_dev) return TCOL_EINVAL;
    HIPCHK(launch_colors(c->ddesc, c->G, c->total_rows, 0, c->stream));
    HIPCHK(launch_mtilde(c->ddesc, c->G, c->total_mt, 0, kFlagMtOut, g, mt_dev, c->stream));
    return TCOL_OK;
}

tcol_status tcol_get_t(tcol_ctx* c, int32_t g, int64_t* t) {
    if (!c || g < 0 || g >= c->G || !t) return TCOL_EINVAL;
    GraphState st;
    HIPCHK(hipMemcpyAsync(&st, c->dstate + g, sizeof(GraphState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    *t = st.t;
    return TCOL_OK;
}

tcol_status tcol_set_t(tcol_ctx* c, int32_t g, int64_t t) {
    if (!c || g < 0 || g >= c->G || t < 0) return TCOL_EINVAL;
    HIPCHK(launch_state(c->ddesc, c->G, 1, g, t, c->stream));
    const tcol_graph_params& p = c->params[g];
    if (c->hdesc[g].vel)
        HIPCHK(hipMemsetAsync(c->hdesc[g].vel, 0, sizeof(float) * (size_t)p.D * p.n * p.k, c->stream));
    return TCOL_OK;
}

tcol_status tcol_get_counters(tcol_ctx* c, int32_t g, int64_t* counts) {
    if (!c || g < 0 || g >= c->G || !counts) return TCOL_EINVAL;
    GraphState st;
    HIPCHK(hipMemcpyAsync(&st, c->dstate + g, sizeof(GraphState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    counts[0] = st.it_nopen;
    counts[1] = st.it_dense;
    counts[2] = st.it_sparse;
    return TCOL_OK;
}

tcol_status tcol_reset(tcol_ctx* c) {
    if (!c) return TCOL_EINVAL;
    HIPCHK(launch_state(c->ddesc, c->G, 0, -1, 0, c->stream));
    return TCOL_OK;
}

tcol_status tcol_set_wait_limit(tcol_ctx* c, int32_t polls) {
    if (!c || polls < 0) return TCOL_EINVAL;
    c->spin_limit = polls == 0 ? kBatchSpinDefault : polls;
    drop_graphs(c);   // the limit is a launch argument of the captured runs
    return TCOL_OK;
}

tcol_status tcol_cancel(tcol_ctx* c) {
    if (!c) return TCOL_EINVAL;
    __atomic_store_n(&c->hcancel[0], 1, __ATOMIC_RELEASE);
    return TCOL_OK;
}

tcol_status tcol_profile(tcol_ctx* c, int32_t steps, int32_t as_only, float* ms) {
    if (!c || steps < 1 || !ms) return TCOL_EINVAL;
    constexpr int NP = TCOL_NPHASES;
    constexpr int NE = 10;
    hipEvent_t ev[NE];
    for (int i = 0; i < NE; ++i) HIPCHK(hipEventCreate(&ev[i]));
    double acc[NP] = {0};
    hipStream_t s = c->stream;
    // the batch launch's phases are timed as the fast schedule's kernels
    const int path = path_of(c) == 3 ? 1 : path_of(c);
    HIPCHK(launch_state(c->ddesc, c->G, 0, -1, 0, s));
    if (path != 0) HIPCHK(launch_colors(c->ddesc, c->G, c->total_rows, 1, s));
    for (int it = 0; it < steps; ++it) {
        HIPCHK(hipEventRecord(ev[0], s));
        if (path == 0) HIPCHK(launch_colors(c->ddesc, c->G, c->total_rows, 1, s));
        HIPCHK(hipEventRecord(ev[1], s));
        if (path != 0)
            HIPCHK(enqueue_prep(c, s));
        else
            HIPCHK(launch_prep(c->ddesc, c->G, c->total_mem, c->prep_lds, 1, 0, 0, 0, 0, s));
        HIPCHK(hipEventRecord(ev[2], s));
        HIPCHK(launch_expand(c->ddesc, c->G, c->total_ex, 1, 0, path != 0 ? 1 : 0, s));
        HIPCHK(hipEventRecord(ev[3], s));
        if (path != 0)
            HIPCHK(enqueue_penalty(c, s));
        else
            HIPCHK(launch_mtilde(c->ddesc, c->G, c->total_mt, 1, 0, -1, nullptr, s));
        HIPCHK(hipEventRecord(ev[4], s));
        if (path == 2)
            HIPCHK(launch_gemm(c->fshape, c->ddesc, c->G, c->total_gm[1], 1, 7, 0, s));
        else
            HIPCHK(launch_gemm(c->shape, c->ddesc, c->G, c->total_gm[0], 1, path == 0 ? 15 : 7 | 32 | 64, 0, s));
        HIPCHK(hipEventRecord(ev[5], s));
        if (path == 1) HIPCHK(enqueue_sparse_add(c, false, s));
        HIPCHK(hipEventRecord(ev[6], s));
        HIPCHK(launch_fitness(c->ddesc, c->G, 1,
                              path == 2 ? kFlagFused : (path == 0 ? kFlagPlainPen : kFlagFoldSparse | kFlagFlipFused),
                              -1, s));
        HIPCHK(hipEventRecord(ev[7], s));
        if (path != 2 && !(path == 1 && c->all_pfuse)) HIPCHK(launch_update_any(c, 1, 0, -1, nullptr, nullptr, s));
        HIPCHK(hipEventRecord(ev[8], s));
        if (path != 2) HIPCHK(launch_advance(c->ddesc, c->G, s));
        HIPCHK(hipEventRecord(ev[9], s));
        HIPCHK(hipEventSynchronize(ev[9]));
        float x[NE - 1];
        for (int i = 0; i + 1 < NE; ++i) HIPCHK(hipEventElapsedTime(&x[i], ev[i], ev[i + 1]));
        // phases: colours, class sizes, expansion, penalty (operand or sparse rows),
        // contraction, fitness, update, advance
        acc[0] += x[0];
        acc[1] += x[1];
        acc[2] += x[2];
        acc[3] += x[3] + x[5];
        acc[4] += x[4];
        acc[5] += x[6];
        acc[6] += x[7];
        acc[7] += x[8];
    }
    for (int i = 0; i < 8; ++i) ms[i] = (float)(acc[i] / steps);
    // the contraction again, `steps` launches back to back on the operands of the last
    // iteration, with the dense penalty pass unless the graphs take the sparse rows in
    // every iteration (its G store is idempotent; the conflict accumulators are cleared
    // after; the operand values may be stale, which does not change the work)
    {
        HIPCHK(hipEventRecord(ev[0], s));
        for (int it = 0; it < steps; ++it) {
            if (path == 2)
                HIPCHK(launch_gemm(c->fshape, c->ddesc, c->G, c->total_gm[1], 1, 7, 0, s));
            else
                HIPCHK(launch_gemm(c->shape, c->ddesc, c->G, c->total_gm[0], 1, path == 0 || c->opt.penalty != 2 ? 15 : 7, 0, s));
        }
        HIPCHK(hipEventRecord(ev[1], s));
        HIPCHK(launch_state(c->ddesc, c->G, 4, -1, 0, s));
        HIPCHK(hipEventSynchronize(ev[1]));
        float x = 0;
        HIPCHK(hipEventElapsedTime(&x, ev[0], ev[1]));
        ms[4] = x / steps;
    }
    tcol_status st = settle(c);
    if (st != TCOL_OK) return st;
    ms[8] = ms[9] = 0.0f;
    if (as_only) {
        HIPCHK(launch_colors(c->ddesc, c->G, c->total_rows, 0, s));
        HIPCHK(launch_prep(c->ddesc, c->G, c->total_mem, c->prep_lds, 0, 0, 0, 0, 0, s));
        HIPCHK(launch_expand(c->ddesc, c->G, c->total_ex, 0, 0, 0, s));
        // A.S alone, then with the G store too (the form of an iteration on the sparse rows: they
        // take the gather, and on the fast path the store is the uint16 counts for the graphs
        // whose row update rides on them; the store is idempotent).  The state is set to an
        // iteration on the sparse rows for this timing (the next iteration's class-size kernel
        // takes the choice again)
        HIPCHK(launch_state(c->ddesc, c->G, 5, -1, 0, s));
        const int forms[2] = {1 | 128, 1 | 4 | 16 | 128 | (path == 1 ? 32 : 0)};
        for (int f = 0; f < 2; ++f) {
            HIPCHK(hipEventRecord(ev[0], s));
            for (int it = 0; it < steps; ++it)
                HIPCHK(launch_gemm(c->shape, c->ddesc, c->G, c->total_gm[0], 0, forms[f], 0, s));
            HIPCHK(hipEventRecord(ev[1], s));
            HIPCHK(launch_state(c->ddesc, c->G, 4, -1, 0, s));
            HIPCHK(hipEventSynchronize(ev[1]));
            float x = 0;
            HIPCHK(hipEventElapsedTime(&x, ev[0], ev[1]));
            ms[8 + f] = x / steps;
        }
    }
    for (int i = 0; i < NE; ++i) hipEventDestroy(ev[i]);
    return TCOL_OK;
}

}  // extern "C"

// Autotuner results of this process, per device and per context signature (the shapes,
// precisions and problems of its graphs and the requested step schedule): a context with
// the same signature on the same device takes the stored options without timing again.
namespace {
std::mutex g_tune_mu;
std::map<std::string, tcol_options> g_tune_cache;

std::string tune_key(const tcol_ctx* c) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    std::string k = "dev" + std::to_string(dev) + "/f" + std::to_string(c->opt.fused ? 1 : 0);
    for (const auto& p : c->params)
        k += "/" + std::to_string(p.n) + "x" + std::to_string(p.k) + "x" + std::to_string(p.D) + "p" +
             std::to_string(p.precision) + "q" + std::to_string(p.problem) + (p.momentum != 0.0f ? "m" : "");
    return k;
}
}  // namespace

extern "C" {

// Time a few steps of each candidate (step schedule, tile shape, penalty mode) and keep the
// fastest.  The weights and counters are restored after every candidate.
tcol_status tcol_autotune(tcol_ctx* c, int32_t* best_bm, int32_t* best_ntw) {
    if (!c) return TCOL_EINVAL;
    const std::string key = tune_key(c);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            const tcol_options keep = c->opt;
            c->opt = it->second;
            tcol_status s = rebuild_schedule(c);
            if (s != TCOL_OK) {
                c->opt = keep;
                rebuild_schedule(c);
                return s;
            }
            const GemmShape& sh = path_of(c) == 2 ? c->fshape : c->shape;
            if (best_bm) *best_bm = sh.bm;
            if (best_ntw) *best_ntw = sh.ntw;
            return TCOL_OK;
        }
    }
    // backups of W and t
    std::vector<float*> backup(c->G, nullptr);
    std::vector<long long> t0(c->G);
    HIPCHK(hipMemcpyAsync(c->hstate, c->dstate, sizeof(GraphState) * c->G, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int g = 0; g < c->G; ++g) {
        const auto& p = c->params[g];
        const size_t bytes = sizeof(float) * (size_t)p.D * p.n * p.k;
        t0[g] = c->hstate[g].t;
        if (hipMalloc((void**)&backup[g], bytes) != hipSuccess) {
            for (auto b : backup) if (b) hipFree(b);
            return TCOL_ENOMEM;
        }
        HIPCHK(hipMemcpyAsync(backup[g], c->hdesc[g].W[0], bytes, hipMemcpyDeviceToDevice, c->stream));
    }
    auto restore = [&]() -> tcol_status {
        for (int g = 0; g < c->G; ++g) {
            const auto& p = c->params[g];
            HIPCHK(hipMemcpyAsync(c->hdesc[g].W[0], backup[g], sizeof(float) * (size_t)p.D * p.n * p.k,
                                  hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(launch_state(c->ddesc, c->G, 1, g, t0[g], c->stream));
        }
        return TCOL_OK;
    };
    // stop rule off while timing
    std::vector<int> stop(c->G);
    for (int g = 0; g < c->G; ++g) {
        stop[g] = c->hdesc[g].stop_on_legal;
        c->hdesc[g].stop_on_legal = 0;
    }
    const tcol_options base = c->opt;
    tcol_options best = base;
    float best_ms = 1e30f;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    std::vector<tcol_options> cands;
    const std::vector<int> paths = base.fused == 0 ? std::vector<int>{0} : std::vector<int>{1, 2};
    {
        // the batch launch, with its own tile, when these graphs can take it
        tcol_options o = base;
        o.fused = 3;
        o.penalty = 0;
        o.tile_bm = o.tile_ntw = 0;
        if (base.fused != 0) cands.push_back(o);
    }
    for (int path : paths)
        for (auto& sh : kShapes) {
            tcol_options o = base;
            o.fused = path;
            o.tile_bm = sh[0];
            o.tile_ntw = sh[1];
            if (path == 2 && tiles_for(c, sh[0], sh[1], 1) <= 0) continue;
            if (path == 0) {
                cands.push_back(o);
                continue;
            }
            // the per-iteration choice (0) and the two fixed routes
            for (int pen : {0, 1, 2}) {
                o.penalty = pen;
                cands.push_back(o);
            }
        }
    const int warm = 2, timed = 6;
    for (auto& o : cands) {
        c->opt = o;
        if (rebuild_schedule(c) != TCOL_OK) continue;
        if (o.fused == 3 && path_of(c) != 3) continue;
        HIPCHK(launch_state(c->ddesc, c->G, 0, -1, 0, c->stream));
        if (run_steps(c, warm) != TCOL_OK) continue;
        HIPCHK(hipEventRecord(e0, c->stream));
        if (run_steps(c, timed) != TCOL_OK) continue;
        HIPCHK(hipEventRecord(e1, c->stream));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        if (settle(c) != TCOL_OK) continue;
        if (restore() != TCOL_OK) break;
        if (ms < best_ms) {
            best_ms = ms;
            best = o;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    for (int g = 0; g < c->G; ++g) c->hdesc[g].stop_on_legal = stop[g];
    c->opt = best;
    tcol_status s = rebuild_schedule(c);
    HIPCHK(launch_state(c->ddesc, c->G, 0, -1, 0, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (auto b : backup) hipFree(b);
    if (s != TCOL_OK) return s;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = c->opt;
    }
    const GemmShape& sh = path_of(c) == 2 ? c->fshape : c->shape;
    if (best_bm) *best_bm = sh.bm;
    if (best_ntw) *best_ntw = sh.ntw;
    return TCOL_OK;
}

}  // extern "C"

// ------------------------------------------------ allocation-free conflicts -----
//
// tcol_conflicts_noalloc keeps every intermediate in `scratch`, a file-scope device array of
// kNoAllocScratch bytes that each device holds from the library's load until the process
// ends.  In host code `scratch` names a host-side stand-in: its device address comes from
// hipGetSymbolAddress, taken once per device with that device current, and only that
// address is handed to kernels.

namespace {

constexpr size_t kNoAllocScratch = TCOL_NOALLOC_SCRATCH_BYTES;
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kNoAllocScratch];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocMaxDevices] = {};

// address of this device's copy of `scratch`, and the one-time set-up of the kernels the call
// launches (LDS attributes), on first use per device
tcol_status noalloc_scratch(int dev, uint8_t** out) {
    if (dev < 0 || dev >= kNoAllocMaxDevices) return TCOL_EHIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            fprintf(stderr, "libtcol: hipGetSymbolAddress(scratch) failed on device %d: %s\n", dev,
                    hipGetErrorString(e));
            return TCOL_EHIP;
        }
        for (int ntw : {4, 6}) {
            const GemmShape sh{kPrecFP4, ntw == 6 ? 128 : 64, ntw, 0};
            if (gemm_prepare(sh) != hipSuccess) return TCOL_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = (uint8_t*)g_scratch_ptr[dev];
    return TCOL_OK;
}

// the conflict pass's buffers inside the scratch array (A.S in fp4 operands, exact for 0/1)
struct NoAllocLayout {
    size_t desc, state, ones, aop, sop, c, V, cT, f2, fcol, feq, f, total;
    int n_pad, rows_S, cs, cTs;
};

NoAllocLayout noalloc_layout(const tcol_graph_params& p) {
    NoAllocLayout L{};
    L.n_pad = round_up(p.n, kPadN);
    L.rows_S = round_up(p.D * p.k, 16) + kSRowSlack;
    L.cs = round_up(p.n, 64);
    L.cTs = round_up(p.D, 8);
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o += align_up(bytes); return at; };
    L.desc = take(sizeof(GraphDev));
    L.state = take(sizeof(GraphState));
    L.ones = take(16);
    L.aop = take((size_t)L.n_pad * op_row_bytes(kPrecFP4, L.n_pad));
    L.sop = take((size_t)L.rows_S * op_row_bytes(kPrecFP4, L.n_pad));
    L.c = take(sizeof(int16_t) * ((size_t)p.D * L.cs + 64));
    L.V = take(sizeof(int32_t) * (size_t)p.D * p.k);
    L.cT = take(sizeof(int16_t) * (size_t)L.cTs * p.n);
    L.f2 = take(sizeof(int32_t) * p.D);
    L.fcol = take(sizeof(int64_t) * p.D);
    L.feq = take(sizeof(int64_t) * p.D);
    L.f = take(sizeof(int64_t) * p.D);
    L.total = o;
    return L;
}

}  // namespace

extern "C" tcol_status tcol_conflicts_noalloc(const tcol_graph_params* p, const uint8_t* A_dev, const float* W_dev,
                                              int16_t* colors_dev, int64_t* f_main_dev, int64_t* f_sec_dev,
                                              void* stream) {
    if (!p || !A_dev || !W_dev) return TCOL_EINVAL;
    const tcol_status ps = check_params(*p);
    if (ps != TCOL_OK) return ps;
    if (p->problem == TCOL_MCOL) return TCOL_EINVAL;
    const NoAllocLayout L = noalloc_layout(*p);
    if (L.total > kNoAllocScratch) {
        fprintf(stderr, "libtcol: tcol_conflicts_noalloc: n = %d, k = %d, D = %d needs %zu bytes of scratch, "
                "more than its fixed %zu\n", p->n, p->k, p->D, L.total, kNoAllocScratch);
        return TCOL_ENOMEM;
    }
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    uint8_t* base = nullptr;
    const tcol_status ss = noalloc_scratch(dev, &base);
    if (ss != TCOL_OK) return ss;
    hipStream_t s = (hipStream_t)stream;

    GraphDev d;
    memset(&d, 0, sizeof(d));
    d.n = p->n;
    d.k = p->k;
    d.D = p->D;
    d.n_pad = L.n_pad;
    d.cs = L.cs;
    d.ncols = p->D * p->k;
    d.rows_S = L.rows_S;
    d.problem = p->problem;
    d.precision = kPrecFP4;
    d.cmax = 1;   // one colour per vertex (multicolouring is rejected above)
    d.c1 = p->n / p->k;
    d.c2 = (p->n % p->k == 0) ? p->n / p->k : p->n / p->k + 1;
    d.ones_dev = (const unsigned long long*)(base + L.ones + 8);
    d.W[0] = const_cast<float*>(W_dev);
    d.Aop = base + L.aop;
    d.Sop[0] = base + L.sop;
    d.c[0] = (int16_t*)(base + L.c);
    d.V[0] = (int32_t*)(base + L.V);
    d.cT = (int16_t*)(base + L.cT);
    d.cTs = L.cTs;
    d.f2 = (int32_t*)(base + L.f2);
    d.fcol = (int64_t*)(base + L.fcol);
    d.feq = (int64_t*)(base + L.feq);
    d.f = (int64_t*)(base + L.f);
    d.st = (GraphState*)(base + L.state);
    const int total_rows = p->D * p->n;
    d.ex_cblocks = expand_blocks(p->D, p->k, L.n_pad);
    const GemmShape sh{kPrecFP4, L.n_pad >= 2048 ? 128 : 64, L.n_pad >= 2048 ? 6 : 4, 0};
    d.gm_tm[0] = L.n_pad / sh.bm;
    d.gm_tn[0] = ceil_div(d.ncols, gemm_bn(sh.ntw));
    GraphDev* gd = (GraphDev*)(base + L.desc);

    // the previous call's contents: everything from the state on starts at zero (operand
    // padding, the slack rows of S^T, the conflict accumulators, the edge count)
    HIPCHK(launch_zero(base + L.state, L.total - L.state, s));
    HIPCHK(launch_put_desc(d, gd, d.st, s));
    // A is packed without its check (its flag word is ignored): the caller vouches for it
    HIPCHK(launch_pack_graph(A_dev, p->n, L.n_pad, kPrecFP4, nullptr, d.Aop, (int*)(base + L.ones),
                             (unsigned long long*)(base + L.ones + 8), s));
    HIPCHK(launch_colors(gd, 1, total_rows, 0, s));
    HIPCHK(launch_prep(gd, 1, p->D, prep_lds(p->k, p->n, 0), 0, 0, 0, 0, 0, s));
    HIPCHK(launch_expand(gd, 1, d.ex_cblocks, 0, 0, 0, s));
    HIPCHK(launch_gemm(sh, gd, 1, d.gm_tm[0] * d.gm_tn[0], 0, 1, 0, s));
    HIPCHK(launch_fitness(gd, 1, 0, kFlagReport, -1, s));
    HIPCHK(launch_copy_report(gd, 0, colors_dev, f_main_dev, f_sec_dev, s));
    return TCOL_OK;
}

// ------------------------------------------------------------- descent driver -

tcol_status tcol_init_weights(float* W_dev, int64_t count, uint64_t seed, double sigma0, void* stream) {
    if (!W_dev || count < 0 || !isfinite(sigma0)) return TCOL_EINVAL;
    HIPCHK(launch_init_weights(W_dev, (long long)count, (unsigned long long)seed, sigma0, (hipStream_t)stream));
    return TCOL_OK;
}

tcol_status tcol_descent(const uint8_t* A_dev, const tcol_graph_params* base, const tcol_descent_options* opt,
                         tcol_descent_result* result, int16_t* colors_dev, void* stream) {
    if (!A_dev || !base || !opt || !result) return TCOL_EINVAL;
    if (base->problem != TCOL_KCOL && base->problem != TCOL_ECP) return TCOL_EINVAL;
    if (opt->k_first < 1 || opt->k_first > kMaxK || opt->k_min < 1 || opt->k_min > opt->k_first ||
        opt->max_steps < 1 || opt->attempts < 1 || !(opt->sigma0 > 0.0) || !isfinite(opt->sigma0))
        return TCOL_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    result->k_best = -1;
    result->k_tried = 0;
    result->attempt_best = -1;
    result->steps_best = 0;
    result->steps_total = 0;
    int16_t* found = nullptr;          // legal colouring of the current attempt
    if (hipMalloc((void**)&found, sizeof(int16_t) * (size_t)std::max(1, base->n)) != hipSuccess) return TCOL_ENOMEM;
    tcol_status rc = TCOL_OK;
    for (int k = opt->k_first; k >= opt->k_min && rc == TCOL_OK; --k) {
        tcol_graph_params p = *base;
        p.k = k;
        p.stop_on_legal = 1;
        rc = check_params(p);
        if (rc != TCOL_OK) break;
        ++result->k_tried;
        bool legal = false;
        for (int r = 0; r < opt->attempts && !legal && rc == TCOL_OK; ++r) {
            const size_t count = (size_t)p.D * p.n * p.k;
            float* W = nullptr;
            if (hipMalloc((void**)&W, sizeof(float) * count) != hipSuccess) {
                rc = TCOL_ENOMEM;
                break;
            }
            const uint64_t seed = opt->seed + 1000003ull * (uint64_t)k + (uint64_t)r;
            rc = tcol_init_weights(W, (int64_t)count, seed, opt->sigma0, s);
            tcol_ctx* c = nullptr;
            if (rc == TCOL_OK) {
                const uint8_t* As[1] = {A_dev};
                float* Ws[1] = {W};
                rc = tcol_init(&c, 1, &p, As, Ws, nullptr, 0, s);
            }
            if (rc == TCOL_OK) {
                int32_t done = 0, legal_d = -1;
                int16_t* outs[1] = {found};
                rc = tcol_step(c, opt->max_steps, &done, &legal_d, outs);
                result->steps_total += done;
                if (rc == TCOL_OK && legal_d >= 0) {
                    legal = true;
                    result->k_best = k;
                    result->attempt_best = r;
                    // the iteration that found the legal member performs no update
                    result->steps_best = done + 1;
                    if (colors_dev &&
                        hipMemcpyAsync(colors_dev, found, sizeof(int16_t) * p.n, hipMemcpyDeviceToDevice, s) != hipSuccess)
                        rc = TCOL_EHIP;
                }
            }
            tcol_destroy(c);
            if (hipStreamSynchronize(s) != hipSuccess && rc == TCOL_OK) rc = TCOL_EHIP;
            hipFree(W);
        }
        if (!legal) break;
    }
    hipFree(found);
    return rc;
}
