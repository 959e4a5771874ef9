// One launch for a run of iterations over a batch of graphs (Algorithm 1, steps 1-4, for
// every graph of a context: the fast schedule with the dense penalty pass).
//
// The launch's work is a queue of items: for each iteration and each phase, every graph's
// items of that phase
//   0  class sizes (one item per member) and the one-hot S^T expansion (Section 3.5),
//   1  group concentration and penalty operand tiles (Section 3.6, eqs. (4)-(6)),
//   2  contraction tiles A.S (+ P.S) with the f_color gather (eqs. (1), (17)),
//   3  fitness and stop rule (Section 3.3),
//   4  softmax straight-through update, smoothing and the next colours (eqs. (8)-(16)),
// in segments ordered by (iteration, phase, graph).  Each block takes the next ticket of a
// device counter when it starts, runs that item and leaves.  Before running it, the block
// waits until every item of the same graph in earlier segments is done (a per-graph count
// of finished items): a graph's phases follow one another while other graphs' phases run
// beside them, with no launch boundary between phases or iterations.  A ticket is only
// taken by a block that is already running and only waits for smaller tickets, so the
// queue drains whatever order the hardware starts blocks in.  Every wait is bounded: it
// gives up after a spin limit the host sets, or when the host's cancel word (pinned host
// memory) is set, and then marks the run aborted; every later block returns at once.
//
// The block bodies are those of the separate kernels (tcol_kernels.hip, tcol_gemm.hip);
// this file is compiled in the same translation unit (tcol_device.hip).
#include "tcol_internal.h"
#include "tcol_launch.h"

namespace tcol {

// one item of the queue: where it starts, whose and which phase it is, and how many items
// of its graph in earlier segments must be done first
struct BatchSegDev {
    int start;
    int g;
    int phase;
    int iter;
    int need;
    int pad[3];
};
static_assert(sizeof(BatchSegDev) == sizeof(BatchSeg), "segment layout");

template <int PREC, int BM, int NTW, int KPL>
__device__ __forceinline__ void batch_item(const GraphDev* __restrict__ gd, int G, const BatchSegDev& S, int idx) {
    extern __shared__ __attribute__((aligned(16))) uint8_t batch_lds[];
    const GraphDev& d = gd[S.g];
    switch (S.phase) {
        case 0: {
            // the iteration's first items also end the previous iteration of the run (the
            // graph's first member block), as the class-size launch of the fast schedule does
            const int adv = S.iter > 0;
            if (idx < d.D) {
                prep_member(gd, G, d.mem_begin + idx, 1, 0, 0, adv);
            } else {
                const int b0 = (idx - d.D) * kBatchExpand, b1 = min(b0 + kBatchExpand, d.ex_cblocks);
                for (int b = b0; b < b1; ++b) expand_block(gd, G, d.ex_begin + b, 1, 0, 1, adv);
            }
            break;
        }
        case 1: {
            int16_t(*ci)[64] = (int16_t(*)[64])batch_lds;
            int16_t(*cj)[64] = (int16_t(*)[64])(batch_lds + sizeof(int16_t) * kMtChunk * 64);
            double(*red)[256] = (double(*)[256])(batch_lds + 2 * sizeof(int16_t) * kMtChunk * 64);
            const int t0 = idx * kBatchMtilde, t1 = min(t0 + kBatchMtilde, d.mt_T * (d.mt_T + 1) / 2);
            for (int t = t0; t < t1; ++t) {
                __syncthreads();
                mtilde_block(gd, G, d.mt_begin + t, 1, kFlagGate, -1, nullptr, ci, cj, red);
            }
            break;
        }
        case 2: {
            int tm, tn;
            local_tile<0>(d, idx, tm, tn);
            gemm_tile<PREC, BM, NTW, 0>(gd, S.g, tm, tn, 1, 7 | 64, 0);
            break;
        }
        case 3:
            fitness_graph(gd, S.g, 1, kFlagFoldSparse, (int*)batch_lds);
            break;
        default: {
            const int end = d.row_begin + d.D * d.n;
            for (int u = 0; u < kBatchRowGroups; ++u) {
                const int row = d.row_begin + (idx * kBatchRowGroups + u) * 16 + (threadIdx.x >> 4);
                if (row < end) update_row<KPL, 1>(gd, G, row, 1, 0, -1, nullptr, nullptr);
            }
            break;
        }
    }
}

template <int PREC, int BM, int NTW, int KPL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_batch_run(
    const GraphDev* __restrict__ gd, int G, const BatchSegDev* __restrict__ segs, int nseg, int total,
    int* __restrict__ ctl, const volatile int* __restrict__ cancel, int spin_limit) {
    extern __shared__ __attribute__((aligned(16))) uint8_t batch_lds[];
    // ctl: [0] abort (kept for the whole tcol_step), then per launch [4] ticket, [5] tickets past
    // the end, [kBatchCtl ...] the done counts of the graphs
    int* abort_flag = ctl;
    int* ticket = ctl + 4;
    int* done = ctl + kBatchCtl;
    volatile int* bc = (volatile int*)batch_lds;   // broadcasts, before the item's phase uses the LDS
    if (threadIdx.x == 0) {
        const int t = atomicAdd(ticket, 1);
        // one item in 256 also reads the host's cancel word (host memory: a slow read)
        if ((t & 255) == 0 && *cancel != 0) atomicExch(abort_flag, 1);
        bc[0] = t;
        bc[1] = __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    // uniform over the block: scalar registers, so the segment and the graph's descriptor
    // fields are read with scalar loads
    const int t = __builtin_amdgcn_readfirstlane(bc[0]);
    const int aborted = __builtin_amdgcn_readfirstlane(bc[1]);
    if (t >= total || aborted) {
        if (threadIdx.x == 0 && t >= total) atomicAdd(ctl + 5, 1);
        return;
    }
    // the segment holding ticket t: the last one starting at or before it
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].start <= t) lo = mid; else hi = mid - 1;
    }
    const BatchSegDev S = segs[lo];
    __syncthreads();   // every wave has read the broadcast
    if (threadIdx.x == 0) {
        // wait for the graph's earlier items: plain polls of the count (no cache maintenance
        // while other blocks compute), then one acquire for the whole block
        int go = 1, spins = 0;
        while (__hip_atomic_load(&done[S.g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < S.need) {
            if ((spins & 63) == 0 &&
                (*cancel != 0 || __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                go = 0;
                break;
            }
            if (++spins > spin_limit) {
                go = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        if (!go) atomicExch(abort_flag, 1);
        // acquire: the writes of the graph's earlier items (other blocks, other XCDs), for
        // every wave of the block (they share this CU's caches).  The fence's cache
        // invalidation is not counted by the compiler's wait tracking, so the wait for it
        // is explicit: the other waves load only after the barrier below.
        __atomic_thread_fence(__ATOMIC_ACQUIRE);
        wait_vm<0>();
        bc[2] = go;
    }
    __syncthreads();
    if (!__builtin_amdgcn_readfirstlane(bc[2])) return;
    batch_item<PREC, BM, NTW, KPL>(gd, G, S, t - S.start);
    // every wave's stores have completed at the barrier; one release then publishes them.
    // The release writes this XCD's L2 back to memory; the compiler does not count that
    // write-back among the operations a wait covers and drops the wait after it.  Without
    // the explicit wait the count can rise while the write-back is still under way, and a
    // waiting item on another XCD then reads stale weights.
    __syncthreads();
    if (threadIdx.x == 0) {
        __atomic_thread_fence(__ATOMIC_RELEASE);
        wait_vm<0>();
        __hip_atomic_fetch_add(&done[S.g], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ------------------------------------------------------------------ dispatch --

#define TCOL_BATCH_KERNELS(X) \
    X(kPrecFP32, 8) X(kPrecBF16, 8) X(kPrecFP8, 8) X(kPrecFP4, 8) \
    X(kPrecFP32, 36) X(kPrecBF16, 36) X(kPrecFP8, 36) X(kPrecFP4, 36)

int batch_kpl(int kmax) {
    const int need = (kmax + 15) / 16;
    if (need <= 8) return 8;
    if (need <= 36) return 36;
    return 0;
}

size_t batch_lds_bytes(int prec, size_t prep_bytes) {
    GemmShape s{prec, kBatchBM, kBatchNTW, 0};
    size_t b = gemm_lds_bytes(s, 0);
    const size_t mt = 2 * sizeof(int16_t) * kMtChunk * 64 + 2 * 256 * sizeof(double);
    if (mt > b) b = mt;
    if (prep_bytes > b) b = prep_bytes;
    return b;
}

hipError_t batch_prepare(int prec, int kpl, int* blocks_per_cu) {
    bool found = false;
    const size_t lds = batch_lds_bytes(prec, 0);
#define TCOL_BATCH_PREP(P, K)                                                                                  \
    if (!found && prec == P && kpl == K) {                                                                     \
        found = true;                                                                                          \
        const void* f = (const void*)k_batch_run<P, kBatchBM, kBatchNTW, K>;                                   \
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);         \
        if (e != hipSuccess) return e;                                                                         \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, 256, lds);                          \
        if (e != hipSuccess) return e;                                                                         \
    }
    TCOL_BATCH_KERNELS(TCOL_BATCH_PREP)
#undef TCOL_BATCH_PREP
    return found ? hipSuccess : hipErrorInvalidValue;
}

hipError_t launch_batch_run(int prec, int kpl, int grid, size_t lds, const GraphDev* gd, int G, const BatchSeg* segs,
                            int nseg, int total, int* ctl, const int* cancel, int spin_limit, hipStream_t s) {
    if (total <= 0 || nseg <= 0) return hipSuccess;
    if (grid <= 0 || lds > 160 * 1024) return hipErrorInvalidValue;
    bool found = false;
#define TCOL_BATCH_LAUNCH(P, K)                                                                               \
    if (!found && prec == P && kpl == K) {                                                                    \
        found = true;                                                                                         \
        k_batch_run<P, kBatchBM, kBatchNTW, K><<<grid, 256, lds, s>>>(                                        \
            gd, G, (const BatchSegDev*)segs, nseg, total, ctl, (const volatile int*)cancel, spin_limit);      \
    }
    TCOL_BATCH_KERNELS(TCOL_BATCH_LAUNCH)
#undef TCOL_BATCH_LAUNCH
    if (!found) return hipErrorInvalidValue;
    const hipError_t e = hipGetLastError();
    return e;
}

}  // namespace tcol
