/*
 * tcol.h -- C ABI of the MI355X (gfx950) population step of TensCol.
 *
 * The method (Goudet, Duval, Hao: "Population-based Gradient Descent Weight
 * Learning for Graph Coloring Problems") keeps D weight tensors W_d (n x k)
 * per graph.  One iteration (Section 3, Algorithm 1, steps 1-4):
 *   1. S = one_hot(argmax(W)) along the colour axis;
 *   2. fitness f_color(S_d) = 1/2 sum(A o S_d S_d^T)   (eq. individual fitness),
 *      plus the equity fitness f_eq for the ECP           (eq. equity fitness);
 *   3. group concentration Mt = sum_d S_d S_d^T           (eq. tildeM) and the
 *      gradient of the global loss                        (eq. global loss gradient)
 *        gS = A.S + nu t grad f_eq + 2 alpha lambda t (A o Mt^(alpha-1)).S
 *             - 2 beta mu t ((J - A) o Mt^(beta-1)).S;
 *   4. straight-through softmax gradient gW = S^ o (gS - (S^ o gS).J)
 *      (eq. tensor gradient), W <- W - eta gW, and W <- W / rho every nb_iter
 *      iterations (eq. smoothing).
 * The loop stops when some member is legal (f = 0, Section 3.3, general scheme).
 *
 * Conventions fixed by this library where the paper leaves a choice:
 *  - argmax ties go to the lowest colour;
 *  - c1 = floor(n/k), c2 = ceil(n/k) in the equity fitness;
 *  - an iteration that finds a legal member stops before its update and
 *    returns the lowest such member;
 *  - smoothing follows the update of iteration t when (t+1) mod nb_iter = 0;
 *  - kappa and varpi sum over ordered pairs; the bonus matrix J - A keeps its
 *    diagonal unless bonus_diag = 0; 0^p = 0.
 *
 * Memory: every pointer named *_dev is a device pointer on the current HIP
 * device.  The caller owns A, W, all outputs and the optional workspace; the
 * library owns only small host state plus, when no workspace is given, the
 * device memory it allocates at init and frees in tcol_destroy.
 *
 * Streams: all device work is enqueued on the stream given at init (a
 * hipStream_t passed as void*; NULL = the default stream).  tcol_step
 * synchronises that stream once, at its end, to fill its host outputs; the
 * other calls are asynchronous.
 *
 * Errors: every call returns a tcol_status; on an error no output is
 * guaranteed.  tcol_status_string gives a static description.
 */
#ifndef TCOL_H
#define TCOL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tcol_status;
enum {
    TCOL_OK = 0,
    TCOL_EINVAL = -1,      /* bad argument (NULL, out-of-range parameter, g out of range) */
    TCOL_ESHAPE = -2,      /* bad n, k or D, or a size beyond the supported maximum */
    TCOL_EGRAPH = -3,      /* A not symmetric, diagonal not zero, or an entry not 0/1 */
    TCOL_EHIP = -4,        /* a HIP runtime call failed */
    TCOL_ENONFINITE = -5,  /* a weight is NaN or infinite */
    TCOL_ENOMEM = -6,      /* device allocation failed or the workspace is too small */
    TCOL_ESTATE = -7,      /* call not valid in the current state */
    TCOL_EABORT = -8       /* a wait of the batch launch gave up (tcol_cancel, or past the
                              limit of tcol_set_wait_limit); the run's weights are unspecified */
};

/* Problem statement.  k-COL is one step of the GCP (Sections 3.1-3.2: fitness =
 * conflicting edges f_color); the ECP adds the equity fitness f_eq to the
 * fitness and nu t f_eq to the loss.  Section 6: k-partitioning replaces every
 * association matrix M by J - M, so the fitness is the number of cut edges
 * |E| - f_color, the group concentration enters the penalty and bonus as
 * D - Mt, and the gradient of the fitness term is -A.S; balanced k-partitioning
 * adds the equity fitness as the ECP does; minimum sum colouring replaces the
 * equity fitness by the colour cost sum_i z_{c(i)} with z_l = l + 1 (colours
 * counted from 0), whose gradient is nu t z_l.  "Main" fitness below means
 * f_color (colouring problems) or the cut (partitioning), "added" fitness f_eq,
 * the colour cost or 0; a member is legal when their sum is 0. */
enum { TCOL_KCOL = 0, TCOL_ECP = 1, TCOL_KPART = 2, TCOL_BKPART = 3, TCOL_MSCP = 4, TCOL_MCOL = 5 };

/* TCOL_MCOL, multicolouring (Section 6): vertex i has a demand c_i (tcol_set_demand; 1 until
 * set) and takes c_i different colours, adjacent vertices sharing none.  Step 1 selects, in
 * each member, the c_i colours of largest weight in w_{d,i} (equal weights: the lower colour
 * first, so c_i = 1 is the argmax); S_d is then multi-hot, M_d = S_d S_d^T counts the colours
 * two vertices share, and f_color = 1/2 sum(A o M_d) (the (edge, shared colour) pairs), Mt,
 * the loss and its gradient keep their tensor forms (eqs. (1), (4)-(7), (17)).  A member is
 * legal when f_color = 0.  Such graphs run the plain step schedule with the dense penalty
 * operand, without momentum, with k <= 1024 and max_demand (below) colours per vertex at
 * most. */

/* Operand precision of the contractions A.S and (penalty).S.  The 0/1
 * operands A and S are exact in every format and accumulate in FP32, so the
 * conflict counts are exact in all four; the penalty operand is rounded to
 * bf16 in TCOL_BF16, TCOL_FP8 and TCOL_FP4 (TCOL_FP8 runs A.S in fp8 e4m3,
 * TCOL_FP4 in fp4 e2m1, both with the penalty product in bf16).  Softmax,
 * gradient and update are FP32. */
enum { TCOL_FP32 = 0, TCOL_BF16 = 1, TCOL_FP8 = 2, TCOL_FP4 = 3 };

/* Parameters of one graph (parameter table of the paper: eta 1e-3, nb_iter 5,
 * rho in {1,2,10,100,200}, alpha 2.5, lambda 1e-5, beta 1.2, mu 1e-6 (GCP) or 0
 * (ECP), nu 0 (GCP) or 1e-5 (ECP)). */
typedef struct {
    int32_t problem;        /* TCOL_KCOL, TCOL_ECP, TCOL_KPART, TCOL_BKPART, TCOL_MSCP or TCOL_MCOL */
    int32_t precision;      /* TCOL_FP32, TCOL_BF16, TCOL_FP8 or TCOL_FP4 */
    int32_t n, k, D;        /* vertices (1..32768), colours (1..4096), members (1..1024) */
    float eta, rho;         /* learning rate > 0; smoothing divisor >= 1 */
    int32_t nb_iter;        /* smoothing period >= 1 */
    float alpha, lambda;    /* penalisation exponent (> 1 when lambda > 0) and weight >= 0 */
    float beta, mu;         /* bonus exponent (> 1 when mu > 0) and weight >= 0 */
    float nu;               /* equity weight >= 0 (ECP) */
    int32_t bonus_diag;     /* 1: bonus matrix J - A includes i = j (literal); 0: excludes it */
    int32_t stop_on_legal;  /* 1: Algorithm 1 stop rule; 0: never stop (timing) */
    float momentum;         /* heavy-ball coefficient gamma in [0, 1) (Section 7: optimiser
                               variants): v <- gamma v + gW, W <- W - eta v, v from zero;
                               0 = the paper's plain step.  With gamma > 0 the epilogue
                               step schedule is not used (the fast one runs instead) */
    int32_t max_demand;     /* TCOL_MCOL: the largest demand c_i (1..8, at most k); other
                               problems: 0 or 1 */
} tcol_graph_params;

/* Execution options of a context. */
typedef struct {
    int32_t fused;          /* step schedule: 0 = plain path (argmax, dense penalty operand,
                               contraction, update as separate kernels every iteration);
                               1 = fast path (default): the update kernel also colours the
                               updated rows, no separate argmax pass (k <= 576, else the plain
                               order); the penalty term as `penalty` selects; a graph whose
                               penalty may take the sparse rows (and takes no heavy-ball steps)
                               gets its row update from the sparse-rows kernel in every
                               iteration, into a second weight buffer that the stop rule
                               accepts or discards, and its A.S counts of the sparse
                               iterations are stored as uint16;
                               2 = epilogue path: the contraction kernel itself applies softmax,
                               gradient, update and the next argmax, into a second weight
                               buffer (k <= 576);
                               3 = batch launch: the fast schedule's work of a whole run of
                               iterations (up to 64) over every graph in ONE kernel launch,
                               whose blocks take items (class sizes and expansion, group
                               concentration tiles, contraction tiles, fitness, row-update
                               groups) from a device queue in ticket order; an item waits
                               until its graph's earlier phases are done, so graphs overlap
                               their phases (Algorithm 1 per graph; a batch of uneven graphs
                               is the use).  It needs the dense penalty pass for every graph
                               (penalty 1, or 0 where the automatic choice keeps it), no
                               heavy-ball steps, no multicolouring, one operand precision and
                               k <= 576; otherwise the fast path runs.  Its contraction tile
                               is 64 x 128 (tile_bm / tile_ntw do not apply).  Waits are
                               bounded (tcol_set_wait_limit) and cancellable (tcol_cancel) */
    int32_t use_graph;      /* 1: replay each step from a captured hipGraph (default) */
    int32_t unroll;         /* steps per captured graph (1..64, default 8) */
    int32_t tile_bm;        /* GEMM rows per block (64, 128 or 256); 0 = default or autotuned */
    int32_t tile_ntw;       /* GEMM 16-column subtiles per wave; the instantiated (tile_bm, tile_ntw)
                               pairs are (64,2) (64,4) (128,4) (128,6) (128,8) (64,9) (128,9)
                               and, with 8 waves, (256,4) (256,6) */
    int32_t penalty;        /* fast and epilogue paths, penalty term P.S with
                               P = 2 alpha lambda t A o Mt^(alpha-1) - 2 beta mu t (J-A) o Mt^(beta-1)
                               (eq. 17, Section 3.8.2): 1 = dense operand pass on MFMA (operand
                               bf16 in the fp4 / fp8 / bf16 modes); 2 = sparse rows in every
                               iteration: with one-hot S_d, (P.S_d)[i, l] is the sum of P_ij over
                               the vertices of colour l in member d, and P_ij = 0 unless j shares
                               i's colour in some member, so each row adds its nonzeros (64-bit
                               fixed-point sums of the FP32 values, exact for the paper's
                               parameters up to n = 4000, rounded once to FP32);
                               0 = choose (default): the sparse rows in the iterations where the
                               rows average at most n class-mates and the dense pass in the
                               others (decided on the device each iteration), the dense pass
                               throughout when 4 D > k or n < 2750, the sparse rows throughout
                               for k-partitioning with n >= 2048 (the dense pass below: the
                               faster route at those sizes); 3 = as 0 without the floors on n.
                               Graphs too large for the sparse kernel's LDS take the dense
                               pass. */
} tcol_options;

typedef struct tcol_ctx tcol_ctx;

/* Static text for a status code. */
const char *tcol_status_string(tcol_status s);

/* Device bytes needed for G graphs with parameters p[G] (for tcol_init's workspace).
 * Errors: TCOL_EINVAL (NULL), TCOL_ESHAPE (sizes out of range). */
tcol_status tcol_workspace_size(int32_t G, const tcol_graph_params *p, size_t *bytes);

/* Create a context for G >= 1 graphs stepped together.
 *   p[G]      parameters per graph (copied);
 *   A_dev[G]  adjacency, n x n uint8 row-major 0/1, symmetric, zero diagonal;
 *             read during this call only (packed copies are kept);
 *   W_dev[G]  weights, D x n x k fp32 row-major; caller-owned, read and
 *             updated in place by tcol_step; must stay valid for the context;
 *   ws_dev    device workspace of ws_bytes >= tcol_workspace_size, or NULL to
 *             let the library allocate it;
 *   stream    hipStream_t (as void*) for all work, NULL = default stream.
 * The iteration counter t of every graph starts at 0.
 * Errors: TCOL_EINVAL, TCOL_ESHAPE, TCOL_EGRAPH (A fails validation),
 *         TCOL_ENOMEM, TCOL_EHIP.  On error *ctx is NULL. */
tcol_status tcol_init(tcol_ctx **ctx, int32_t G, const tcol_graph_params *p,
                      const uint8_t *const *A_dev, float *const *W_dev,
                      void *ws_dev, size_t ws_bytes, void *stream);

/* Multicolouring demands of graph g (a TCOL_MCOL graph): demand (host, n int32) c_i in
 * 1..max_demand.  Copied; takes effect from the next call.  Synchronises the stream.
 * Errors: TCOL_EINVAL (not a TCOL_MCOL graph, NULL, a demand out of range), TCOL_EHIP. */
tcol_status tcol_set_demand(tcol_ctx *ctx, int32_t g, const int32_t *demand);

/* The selection of step 1 for graph g at its current W: sel_dev (device, D*n*max_demand int16,
 * [d][i][s]) receives the s-th colour of vertex i in member d in decreasing weight (ties: lower
 * colour first), -1 past the vertex's demand; for other problems max_demand is 1 and this is
 * the argmax colouring.  Asynchronous.  Errors: TCOL_EINVAL, TCOL_EHIP. */
tcol_status tcol_selection(tcol_ctx *ctx, int32_t g, int16_t *sel_dev);

/* Change execution options (before or between tcol_step calls). */
tcol_status tcol_set_options(tcol_ctx *ctx, const tcol_options *opt);
tcol_status tcol_get_options(tcol_ctx *ctx, tcol_options *opt);

/* Run up to max_steps iterations of Algorithm 1 on every graph (steps 1-4;
 * a graph whose population holds a legal member stops before that
 * iteration's update when stop_on_legal = 1).
 *   steps_done (host, may be NULL): largest number of updates any graph made;
 *   legal_d (host [G], may be NULL): lowest legal member d* of each graph in
 *     the iteration where it stopped, or -1;
 *   colors_out_dev ([G] device pointers to n int16 each, may be NULL, entries
 *     may be NULL): colouring S_{d*} of each graph that stopped.
 * Synchronises the stream once.  Errors: TCOL_ENONFINITE (some weight is not
 * finite; the affected graph stops without updating), TCOL_EHIP, TCOL_EINVAL. */
tcol_status tcol_step(tcol_ctx *ctx, int32_t max_steps, int32_t *steps_done, int32_t *legal_d,
                      int16_t *const *colors_out_dev);
/* (For a TCOL_MCOL graph colors_out_dev[g] receives n * max_demand int16, [i][s], -1 padded.) */

/* Steps 1-2 only, on the current W of graph g (W unchanged, t unchanged):
 *   colors_dev (D*n int16, may be NULL) argmax colours c_d(i);
 *   f_main_dev (D int64, may be NULL) main fitness per member: f_color, computed
 *              from the contraction A.S as 1/2 sum_i (A.S_d)[i, c_d(i)], or for
 *              partitioning the cut |E| - f_color;
 *   f_sec_dev  (D int64, may be NULL) added fitness per member: f_eq (ECP,
 *              balanced partitioning), the colour cost (minimum sum colouring)
 *              or 0.
 * Asynchronous.  Errors: TCOL_EINVAL. */
tcol_status tcol_conflicts(tcol_ctx *ctx, int32_t g, int16_t *colors_dev, int64_t *f_main_dev,
                           int64_t *f_sec_dev);

/* Loss and gradients of graph g at its current W and t (no update):
 *   loss_dev  (5 doubles, may be NULL): L, sum of the main fitness, sum of the
 *             added fitness, kappa, varpi (eq. global loss, with Mt -> D - Mt
 *             in kappa and varpi for partitioning; FP64 reduction on the GPU);
 *   gradS_dev (D*n*k fp32, may be NULL): gradient of L with respect to S;
 *   gradW_dev (D*n*k fp32, may be NULL): straight-through gradient with respect to W.
 * Asynchronous.  Errors: TCOL_EINVAL. */
tcol_status tcol_loss_grad(tcol_ctx *ctx, int32_t g, double *loss_dev, float *gradS_dev,
                           float *gradW_dev);

/* Class-conflict matrices of graph g at its current W: C_dev (D*k*k int32, [d][l][l'])
 * receives S_d^T A S_d, the number of ordered pairs (i, j) with a_ij = 1, c_d(i) = l and
 * c_d(j) = l' (the edges between colour classes l and l', twice the edges inside class l
 * on the diagonal; its trace is 2 f_color(S_d), Section 3.5 eq. (1) with M_d = S_d S_d^T).
 * Computed as S_d^T (A.S_d): the contraction A.S (stored to G), then an FP32 MFMA
 * contraction over the vertices with the one-hot S_d^T; exact (integers below 2^24).  For
 * partitioning the same matrix of the member's groups.  Asynchronous; overwrites the
 * context's G (the next tcol_step recomputes it).  Errors: TCOL_EINVAL, TCOL_EHIP. */
tcol_status tcol_class_conflicts(tcol_ctx *ctx, int32_t g, int32_t *C_dev);
/* (TCOL_MCOL graphs: TCOL_EINVAL.) */

/* Group concentration matrix Mt (n*n int32, row-major) of graph g at its
 * current W (eq. tildeM).  Asynchronous.  Errors: TCOL_EINVAL. */
tcol_status tcol_mtilde(tcol_ctx *ctx, int32_t g, int32_t *mt_dev);

/* Iteration counter of graph g (checkpoint / resume: the state is W and t).
 * tcol_set_t also clears the graph's momentum velocity (a resumed run restarts
 * the heavy-ball state from zero).  tcol_get_t synchronises the stream. */
tcol_status tcol_get_t(tcol_ctx *ctx, int32_t g, int64_t *t);
tcol_status tcol_set_t(tcol_ctx *ctx, int32_t g, int64_t t);

/* Clear the "stopped" state of every graph so tcol_step continues (for
 * example after the caller changed k or re-initialised W, or after a
 * TCOL_ENONFINITE stop once the caller has restored finite weights). */
tcol_status tcol_reset(tcol_ctx *ctx);

/* Iterations of graph g evaluated since tcol_init (every tcol_step iteration that reached the
 * fitness, the stopping one included; tcol_profile's iterations count too), split by how
 * the penalty product of eq. (17) was taken (Section 3.8.2):
 *   counts[0]  lambda t = mu t = 0, no penalty product (t = 0, or lambda = mu = 0);
 *   counts[1]  the dense operand pass of the contraction (the plain schedule always);
 *   counts[2]  the sparse rows (tcol_options.penalty).
 * counts: host array of 3 int64.  Synchronises the stream.  Errors: TCOL_EINVAL, TCOL_EHIP. */
tcol_status tcol_get_counters(tcol_ctx *ctx, int32_t g, int64_t *counts);

/* Autotuner of the step for this context's graphs: times a few steps of every
 * candidate on the context's stream and keeps the fastest in the options.  The
 * candidates are every instantiated tile shape under the plain schedule (when
 * the options ask for it, fused = 0), else under the fast and the epilogue
 * schedules, each with the per-iteration penalty choice and the two fixed
 * penalty routes (tcol_options.penalty 0, 1, 2).  W and t are restored after
 * every candidate (the trial iterations count in tcol_get_counters).  The
 * result is cached for the process per device and per context signature (n, k,
 * D, precision, problem and momentum of every graph, and whether the plain
 * schedule was asked for): a later call on a context with the same signature
 * applies the cached options without timing.  *best_bm / *best_ntw (host, may
 * be NULL) receive the chosen tile.  Allocates a device copy of each W for the
 * duration of the call.  Errors: TCOL_EINVAL, TCOL_ENOMEM, TCOL_EHIP. */
tcol_status tcol_autotune(tcol_ctx *ctx, int32_t *best_bm, int32_t *best_ntw);

/* Batch launch (tcol_options.fused = 3): the number of polls a waiting item makes before it
 * gives up (each poll sleeps about 50 ns and reads device memory); 0 restores the default
 * (about 4 million polls: seconds).  A run whose wait gave up returns TCOL_EABORT from
 * tcol_step, after every block of the launch has exited.  Drops the captured step graphs (the
 * limit is a launch argument).  For callers that want runs cut short, e.g. tests of the
 * abort path with a tiny limit.  Errors: TCOL_EINVAL (NULL, polls < 0). */
tcol_status tcol_set_wait_limit(tcol_ctx *ctx, int32_t polls);

/* Batch launch: ask a running tcol_step to give up.  Sets a word in pinned host memory that
 * the launch's waits poll; a waiting item then marks the run aborted and every later item
 * returns at once, so the call in progress returns TCOL_EABORT.  Safe to call from another
 * host thread while tcol_step runs; tcol_step clears the word when it starts.  No effect on
 * the other schedules.  Errors: TCOL_EINVAL. */
tcol_status tcol_cancel(tcol_ctx *ctx);

/* Measurement utility.  Runs `steps` iterations of every graph eagerly (no
 * captured graph) with HIP events around each kernel on the context's stream
 * and writes the average milliseconds per iteration of each phase to
 * ms[TCOL_NPHASES]: 0 argmax colours, 1 class sizes, 2 one-hot S expansion,
 * 3 penalty (group concentration + dense operand, or the sparse rows, which on
 * the fast path run after the contraction and add their rows to G, or for the
 * graphs whose row update rides on them, update the rows themselves),
 * 4 contraction A.S (+ dense penalty pass)
 * with fitness gather and, on the fused path, the update epilogue,
 * 5 fitness / stop rule, 6 softmax straight-through update (the separate row
 * update kernel; near zero on the fast path when every graph's update rides on
 * the sparse rows), 7 counter advance.  Phase 4 is timed separately as `steps` contraction
 * launches back to back on the operands of the last iteration (one event pair,
 * so launch gaps do not count), with the f_color gather and the dense penalty
 * pass unless penalty = 2.  When as_only is non-zero it then also times `steps`
 * back-to-back launches of the contraction restricted to the A.S pass (no
 * gather, no store; W unchanged) into ms[8], and `steps` launches of the A.S
 * pass with the store of G (the form the contraction takes on the fast
 * schedule in iterations whose penalty the sparse rows take, which then gather
 * f_color themselves: the uint16 counts for graphs whose row update rides on
 * the sparse rows) into ms[9]; otherwise ms[8] = ms[9] = 0.  Synchronises
 * the stream.
 * Errors: TCOL_EINVAL, TCOL_EHIP. */
#define TCOL_NPHASES 10
tcol_status tcol_profile(tcol_ctx *ctx, int32_t steps, int32_t as_only, float *ms);

/* Measurement utility, no context: the achievable MFMA throughput of the current
 * device for one operand type (precision as in tcol_graph_params: the fp4 / fp8
 * 16x16x128 scaled form, bf16 16x16x32 or fp32 16x16x4), from `iters` rounds of
 * eight dependent-chain MFMAs per wave on register operands over every CU
 * (32 waves per CU, no memory traffic), timed with HIP events on a private
 * stream after a short warm-up.  Writes TFLOP/s (dense, 2 m n k per
 * instruction) to *tflops (host).  Synchronises its stream; allocates no
 * device memory.  Errors: TCOL_EINVAL (NULL, iters < 1, unknown precision),
 * TCOL_EHIP. */
tcol_status tcol_mfma_peak(int32_t precision, int32_t iters, double *tflops);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): tcol_conflicts without a context.  Steps
 * 1-2 for one graph with parameters p (p->problem selects the fitness; p->precision is
 * ignored: the contraction A.S runs in fp4 operands, exact for 0/1 in every format):
 *   A_dev       n x n uint8 row-major 0/1, symmetric, zero diagonal (not checked here:
 *               nonzero entries count as 1);
 *   W_dev       D x n x k fp32 weights (read only);
 *   colors_dev, f_main_dev, f_sec_dev   as tcol_conflicts (each may be NULL).
 * Every intermediate lives in one static device array of TCOL_NOALLOC_SCRATCH_BYTES that
 * each device holds from the library's load until the process ends; the call allocates
 * nothing, launches kernels only on `stream` (hipStream_t as void*, NULL = default) and
 * does not synchronise, so it may be captured into a graph.  Calls on the same device share
 * that array and keep its last contents: calls that may overlap on one device (different
 * streams, or host threads) race and must be ordered by the caller.  The outputs equal
 * tcol_conflicts' for the same A, W and problem.
 * Errors: TCOL_EINVAL (NULL A_dev or W_dev, bad parameters, TCOL_MCOL), TCOL_ESHAPE, TCOL_ENOMEM (the
 * graph needs more scratch than the array holds, about n = 4000 with D k = 8960 at most),
 * TCOL_EHIP. */
#define TCOL_NOALLOC_SCRATCH_BYTES (32u << 20)
tcol_status tcol_conflicts_noalloc(const tcol_graph_params *p, const uint8_t *A_dev, const float *W_dev,
                                   int16_t *colors_dev, int64_t *f_main_dev, int64_t *f_sec_dev, void *stream);

/* Release the context (and the workspace it allocated).  NULL is ignored. */
void tcol_destroy(tcol_ctx *ctx);

/* Initial weights W ~ N(0, sigma0^2) (Section 3.2: sigma0 is their standard
 * deviation, 0.01 in the parameter table), written to W_dev[0 .. count) on the
 * device: Philox4x32-10 with key = seed and counter block b = (b mod 2^32,
 * b / 2^32, 1, 0) gives two 53-bit uniforms u1 = ((w0 >> 5) 2^26 + (w1 >> 6) + 1)
 * 2^-53 and u2 (from w2, w3), and Box-Muller in FP64 the normals
 * sqrt(-2 ln u1) cos(2 pi u2) and sqrt(-2 ln u1) sin(2 pi u2) for entries 2b and
 * 2b + 1, times sigma0, rounded to fp32.  Asynchronous on `stream`.
 * Errors: TCOL_EINVAL (NULL W_dev, count < 0, sigma0 not finite), TCOL_EHIP. */
tcol_status tcol_init_weights(float *W_dev, int64_t count, uint64_t seed, double sigma0, void *stream);

/* Colour-count descent (Sections 1 and 3: the GCP, and likewise the ECP, is
 * approached by solving k-COL (or k-ECP) for decreasing k, each legal k being
 * an upper bound).  Starting from k = k_first, each k gets up to `attempts`
 * runs of at most max_steps iterations, attempt r from fresh weights drawn by
 * tcol_init_weights with seed + 1000003 k + r; a run stops at its first legal
 * member.  The descent moves to k - 1 after a legal colouring and ends at the
 * first k none of whose attempts finds one, or below k_min. */
typedef struct {
    int32_t k_first;        /* first number of colours tried (1..4096) */
    int32_t k_min;          /* smallest k tried (1..k_first) */
    int32_t max_steps;      /* iteration budget of one attempt (>= 1) */
    int32_t attempts;       /* runs per k (>= 1) */
    uint64_t seed;          /* base seed of the initial weights */
    double sigma0;          /* standard deviation of the initial weights (> 0) */
} tcol_descent_options;

typedef struct {
    int32_t k_best;         /* smallest k with a legal colouring found, or -1 */
    int32_t k_tried;        /* number of k values tried */
    int32_t attempt_best;   /* attempt that found the k_best colouring */
    int32_t steps_best;     /* iterations that attempt took (the legal one included) */
    int64_t steps_total;    /* iterations over all attempts */
} tcol_descent_result;

/* Run the descent on one graph (problems TCOL_KCOL and TCOL_ECP).  A_dev: n x n
 * row-major 0/1 (as tcol_init);
 * base: the graph's parameters (k and stop_on_legal are overridden; D,
 * problem, precision and the method's parameters are kept); opt: as above.
 * On return *result (host) holds the outcome and colors_dev (device, n int16,
 * may be NULL) the legal colouring with k_best colours when one was found.
 * The call allocates the weights and the workspace of each run on the device
 * and frees them before it returns; it synchronises `stream`.
 * Errors: TCOL_EINVAL, TCOL_ESHAPE, TCOL_EGRAPH, TCOL_ENOMEM, TCOL_EHIP and
 * TCOL_ENONFINITE (as tcol_init / tcol_step). */
tcol_status tcol_descent(const uint8_t *A_dev, const tcol_graph_params *base, const tcol_descent_options *opt,
                         tcol_descent_result *result, int16_t *colors_dev, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TCOL_H */
