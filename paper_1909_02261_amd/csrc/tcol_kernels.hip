// gfx950 kernels of the TensCol population step other than the MFMA contraction:
// graph validation and packing, argmax colouring, class sizes, one-hot S^T
// expansion, group concentration with the penalty operand, fitness and stop
// rule, softmax straight-through update, loss reduction, state updates.
//
// Every kernel takes the descriptor array of all graphs of a context and a
// flattened work index, so one launch serves a batch of graphs of uneven sizes.
#include "tcol_internal.h"
#include "tcol_launch.h"

#include <math.h>

namespace tcol {

// ---------------------------------------------------------------- helpers ----

__device__ inline uint16_t f32_to_bf16_rne(float x) {
    // round to nearest even on the upper 16 bits (inputs here are finite)
    uint32_t u = __float_as_uint(x);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}

__device__ inline bool finite_f(float x) { return (__float_as_uint(x) & 0x7F800000u) != 0x7F800000u; }

// 1.0 in each operand format
__device__ inline uint32_t one_bits(int prec) {
    return prec == kPrecFP32 ? 0x3F800000u : (prec == kPrecBF16 ? 0x3F80u : 0x38u);
}

__device__ inline int graph_of_row(const GraphDev* gd, int G, int w) {
    return find_graph(gd, G, w, [](const GraphDev& x) { return x.row_begin; });
}

// ---------------------------------------------------- shared device helpers --

__device__ inline bool pen_active(const GraphDev& d, const GraphState* st) {
    const float tf = (float)st->t;
    return (d.lambda * tf != 0.0f) || (d.mu * tf != 0.0f);
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// equal 16-bit halves of a and b among those whose top bit is set in `valid`
// (0x8000 for the low half, 0x80000000 for the high half): a half of a ^ b is zero
// exactly when subtracting one inside that half sets its top bit while the half
// itself does not have it set (colours are < 2^15)
__device__ inline int equal_halves_in(uint32_t a, uint32_t b, uint32_t valid) {
    const uint32_t x = a ^ b;
    u16x2 h = __builtin_bit_cast(u16x2, x);
    const u16x2 one = {1, 1};
    const uint32_t y = __builtin_bit_cast(uint32_t, (u16x2)(h - one));
    return __builtin_popcount(y & ~x & valid);
}

// global-address-space views: loads through them are not ordered against LDS
// operations (a flat pointer may alias LDS, which pins every flat load behind
// the LDS atomics and barriers before it)
template <typename T>
__device__ inline const __attribute__((address_space(1))) T* gview(const T* p) {
    return (const __attribute__((address_space(1))) T*)p;
}
typedef unsigned int u32x4n __attribute__((ext_vector_type(4)));
// order this wave's LDS accesses across lanes (LDS executes a wave's operations in issue order)
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}
// 16-byte global load (p 16-byte aligned)
__device__ inline u32x4n gload16(const void* p) { return *(const __attribute__((address_space(1))) u32x4n*)p; }

// ------------------------------------------------------ validation, packing --

// Checks A (n x n, row-major 0/1, symmetric, zero diagonal) and writes the
// zero-padded byte copy A8 (unless A8 is null) and the operand copy Aop ([n_pad][n_pad];
// in fp4 two entries per byte, the lower column in the low nibble, 1.0 = 0x2).
__global__ __launch_bounds__(256) void k_pack_graph(const uint8_t* __restrict__ A, int n, int n_pad, int prec,
                                                    uint8_t* __restrict__ A8, void* __restrict__ Aop,
                                                    int* __restrict__ bad, unsigned long long* __restrict__ ones) {
    __shared__ unsigned int wcount[4];
    const long long total = (long long)n_pad * n_pad;
    unsigned int count = 0;   // ones of A seen by this thread (2 |E| over all threads of a valid graph)
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e / n_pad), j = (int)(e - (long long)i * n_pad);
        uint8_t a = 0;
        if (i < n && j < n) {
            a = A[(size_t)i * n + j];
            uint8_t b = A[(size_t)j * n + i];
            if (a > 1 || a != b || (i == j && a != 0)) atomicOr(bad, 1);
            a = a ? 1 : 0;
        }
        count += a;
        if (A8) A8[e] = a;
        if (prec == kPrecFP32)
            ((float*)Aop)[e] = a ? 1.0f : 0.0f;
        else if (prec == kPrecBF16)
            ((uint16_t*)Aop)[e] = a ? 0x3F80 : 0;
        else if (prec == kPrecFP8)
            ((uint8_t*)Aop)[e] = a ? 0x38 : 0;
        else if ((j & 1) == 0) {
            // the even column writes the byte of the pair (n_pad is even)
            const uint8_t a1 = (i < n && j + 1 < n) ? (A[(size_t)i * n + j + 1] ? 1 : 0) : 0;
            ((uint8_t*)Aop)[e >> 1] = (uint8_t)((a ? 0x2 : 0) | (a1 ? 0x20 : 0));
        }
    }
    // one atomic per block
    for (int sh = 32; sh >= 1; sh >>= 1) count += __shfl_xor(count, sh);
    if ((threadIdx.x & 63) == 0) wcount[threadIdx.x >> 6] = count;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long c = (unsigned long long)wcount[0] + wcount[1] + wcount[2] + wcount[3];
        if (c) atomicAdd(ones, c);
    }
}

// ------------------------------------------------------------ step 1 -----------

// Multicolouring, step 1 for row r = (member m, vertex i): the dem[i] colours of largest weight,
// one after the other (each the argmax of the colours not yet taken, lowest l on ties), into
// sel[m][s][i] for s < dem[i] and -1 for the other slots; slot 0 also into c[pS].  16 lanes per
// row; lane l16 keeps a bit per colour l16 + 16 q it holds that has been taken (k <= 1024).
__device__ inline void select_row(const GraphDev& d, GraphState* st, int r, const float* w, int l16) {
    const int k = d.k, n = d.n, CM = d.cmax;
    const int m = r / n, i = r - m * n;
    const int ci = d.dem[i];
    int bad = 0;
    for (int l = l16; l < k; l += 16)
        if (!finite_f(w[l])) bad = 1;
    for (int sh = 8; sh >= 1; sh >>= 1) bad |= __shfl_xor(bad, sh, 16);
    if (bad) {
        if (l16 == 0) {
            atomicExch(&st->error, -5);
            atomicExch(&st->stopped, 1);
            d.c[st->pS][(size_t)m * d.cs + i] = 0;
        }
        return;
    }
    unsigned long long taken = 0;
    for (int sl = 0; sl < CM; ++sl) {
        float best = -INFINITY;
        int bi = 0x7FFFFFFF;
        int q = 0;
        for (int l = l16; l < k; l += 16, ++q)
            if (!((taken >> q) & 1ull) && w[l] > best) {
                best = w[l];
                bi = l;
            }
        for (int sh = 8; sh >= 1; sh >>= 1) {
            const float ob = __shfl_xor(best, sh, 16);
            const int oi = __shfl_xor(bi, sh, 16);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        const int pick = (sl < ci && bi < k) ? bi : -1;
        if (pick >= 0 && (pick & 15) == l16) taken |= 1ull << (pick >> 4);
        if (l16 == 0) {
            d.sel[((size_t)m * CM + sl) * d.cs + i] = (int16_t)pick;
            if (sl == 0) d.c[st->pS][(size_t)m * d.cs + i] = (int16_t)pick;
        }
    }
}

// c_d(i) = argmax_l W[d,i,l], lowest l on ties; 16 lanes per row.
__global__ __launch_bounds__(256) void k_colors(const GraphDev* __restrict__ gd, int G, int total_rows,
                                                int honor_stop) {
    const int l16 = threadIdx.x & 15;
    const int row = blockIdx.x * 16 + (threadIdx.x >> 4);
    if (row >= total_rows) return;
    const GraphDev& d = gd[graph_of_row(gd, G, row)];
    GraphState* st = d.st;
    if (honor_stop && st->stopped) return;
    const int r = row - d.row_begin;
    const float* w = d.W[st->pW] + (size_t)r * d.k;
    if (d.cmax > 1) {
        select_row(d, st, r, w, l16);
        return;
    }
    float best = -INFINITY;
    int bi = 0x7FFFFFFF;
    int bad = 0;
    for (int l = l16; l < d.k; l += 16) {
        float x = w[l];
        if (!finite_f(x)) bad = 1;
        if (x > best) { best = x; bi = l; }
    }
    for (int m = 8; m >= 1; m >>= 1) {
        float ob = __shfl_xor(best, m, 16);
        int oi = __shfl_xor(bi, m, 16);
        int obad = __shfl_xor(bad, m, 16);
        bad |= obad;
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (l16 == 0) {
        if (bad || bi >= d.k) {
            bi = 0;
            atomicExch(&st->error, -5);
            atomicExch(&st->stopped, 1);
        }
        const int m = r / d.n, i = r - m * d.n;
        d.c[st->pS][(size_t)m * d.cs + i] = (int16_t)bi;
    }
}

// Per-iteration penalty choice of graphs on the sparse rows (ps_mode 2): row i has at
// most sum_d |class of c_d(i)| nonzeros in P, and over all rows that is
// w = sum_d sum_l #V_{d,l}^2.  While its average over the rows stays within n the
// iteration takes the sparse rows; beyond (the population collapsing into a few large
// classes) the dense pass, whose cost does not depend on the classes.  Partitioning
// keeps the sparse rows: its operand over D - Mt has nonzeros wherever Mt < D, so its
// rows are dense anyway and the sparse kernel is the faster on them.  Returns pdense.
__device__ inline int penalty_choice(const GraphDev& d, long long w) {
    // n: on k-colouring of G(4000, .5) with k = 280, D = 32 (fp4) the step took 0.326 ms against
    // 0.334 (0.4 n), 0.324 (1.5 n), 0.330 (2 n), 0.340 (3 n)
    return d.ps_mode == 2 && !prob_partition(d.problem) && w > (long long)d.n * d.n ? 1 : 0;
}

// Class sizes #V_{d,l} of member d, its added fitness (equity or colour cost) and
// the vertex-major copy of its colours.
// For a graph on the sparse penalty also the member's vertices grouped by colour
// (counting sort) and, for each vertex, the start and size of its class; with `decide`
// the last of the graph's member blocks then takes the iteration's penalty choice
// (penalty_choice).  One block per member.
// Dynamic LDS: k counts, and with the class lists 4 k per-wave cursors, k class starts
// and n entries.
// block b of the S^T expansion (the expansion kernel's body; the fast path runs it in
// extra blocks of the class-size launch, since both read only the colours)
// (adv: the launch also ends the previous iteration, so a pending non-finite update counts as
// a stop)
__device__ __forceinline__ void expand_block(const GraphDev* __restrict__ gd, int G, int b, int honor_stop, int next, int gate,
                             int adv);

// end of an iteration for a running graph: t <- t + 1, and a non-finite weight from the
// update stops the graph with an error
__device__ inline void advance_graph(GraphState* st) {
    if (st->stopped) return;
    st->t += 1;
    st->steps_done += 1;
    if (st->next_bad) {
        st->error = -5;
        st->stopped = 1;
    }
}

constexpr int kPrepScratch = 288;   // words of the class-size block's LDS scratch

// the class-size kernel's block for member `mem` (flattened over the graphs)
constexpr int kPrepBatch = 8;   // colours loaded per lane before the class-size atomics use them

__device__ __forceinline__ void prep_member(const GraphDev* __restrict__ gd, int G, int mem, int honor_stop, int next, int decide,
                            int advance_prev) {
    // dynamic LDS (prep_lds): a scratch of kPrepScratch words (the scan's run sums, two
    // four-wave reductions, the ticket result), then the counts and class lists
    extern __shared__ int prep_dyn[];
    int* part = prep_dyn;                                     // [257]
    long long* fsum = (long long*)(prep_dyn + 260);           // [4]
    long long* qsum = fsum + 4;                               // [4]
    int* last_block_p = prep_dyn + 276;
    int* prep_sh = prep_dyn + kPrepScratch;
    const GraphDev& d = gd[find_graph(gd, G, mem, [](const GraphDev& x) { return x.mem_begin; })];
    GraphState* st = d.st;
    // Whether the graph is stopped for this iteration, read before anything in this launch
    // writes the state: advance_graph below can only turn `stopped` on, and exactly when
    // next_bad is set, so every thread of every member block (and of the expansion blocks)
    // takes the same decision whether it reads `stopped` before or after that write.  A
    // graph's member blocks therefore all run or all return, and the ticket of the penalty
    // choice below counts all of them.
    const bool stop_now = honor_stop && (st->stopped || (advance_prev && st->next_bad));
    // the previous iteration's end (its own launch otherwise), by the graph's first member
    // block: nothing in this launch reads t
    if (advance_prev && mem == d.mem_begin && threadIdx.x == 0) advance_graph(st);
    if (stop_now) return;
    const int p = next ? st->pS ^ 1 : st->pS;
    const int m = mem - d.mem_begin;
    const int k = d.k, n = d.n, tid = threadIdx.x;
    const int16_t* __restrict__ c = d.c[p] + (size_t)m * d.cs;
    int16_t* __restrict__ cT = d.cT;
    const size_t cTs = d.cTs;
    int* cnt = prep_sh;
    const bool lists = d.psparse != 0;              // uniform over the block
    // with the class lists each wave counts its own quarter of the vertices
    constexpr int NW = 4;
    const int wv = tid >> 6, lane = tid & 63;
    const int Q = ((n + NW - 1) / NW + 63) & ~63;
    int* cw = prep_sh + k;                          // [NW][k]
    for (int l = tid; l < k; l += 256) cnt[l] = 0;
    if (lists)
        for (int l = tid; l < NW * k; l += 256) cw[l] = 0;
    __syncthreads();
    // the vertex loops load kPrepBatch colours per lane before using any of them (one round
    // of load latency per batch instead of one per vertex)
    if (lists) {
        const int e = min(n, (wv + 1) * Q);
        for (int i0 = wv * Q + lane; i0 < e; i0 += 64 * kPrepBatch) {
            int16_t xs[kPrepBatch];
#pragma unroll
            for (int u = 0; u < kPrepBatch; ++u) xs[u] = i0 + 64 * u < e ? gview(c)[i0 + 64 * u] : (int16_t)0;
#pragma unroll
            for (int u = 0; u < kPrepBatch; ++u) {
                const int i = i0 + 64 * u;
                if (i < e) {
                    atomicAdd(&cnt[xs[u]], 1);
                    atomicAdd(&cw[wv * k + xs[u]], 1);
                    cT[(size_t)i * cTs + m] = xs[u];
                }
            }
        }
    } else if (d.cmax > 1) {
        // multicolouring: every selected colour of the vertex counts in its class
        for (int i = tid; i < n; i += 256) {
            for (int sl = 0; sl < d.cmax; ++sl) {
                const int16_t x = d.sel[((size_t)m * d.cmax + sl) * d.cs + i];
                if (x >= 0) atomicAdd(&cnt[x], 1);
            }
            cT[(size_t)i * cTs + m] = gview(c)[i];
        }
    } else {
        for (int i0 = tid; i0 < n; i0 += 256 * kPrepBatch) {
            int16_t xs[kPrepBatch];
#pragma unroll
            for (int u = 0; u < kPrepBatch; ++u) xs[u] = i0 + 256 * u < n ? gview(c)[i0 + 256 * u] : (int16_t)0;
#pragma unroll
            for (int u = 0; u < kPrepBatch; ++u) {
                const int i = i0 + 256 * u;
                if (i < n) {
                    atomicAdd(&cnt[xs[u]], 1);
                    cT[(size_t)i * cTs + m] = xs[u];
                }
            }
        }
    }
    __syncthreads();
    int32_t* V = d.V[p] + (size_t)m * k;
    for (int l = tid; l < k; l += 256) V[l] = cnt[l];
    // added fitness of the member from the counts: f_eq = sum_l min(|#V - c1|, |#V - c2|),
    // or the colour cost sum_l (l + 1) #V_l (the fitness kernel of this iteration reads it)
    if (prob_added(d.problem)) {
        const int c1 = d.c1, c2 = d.c2;
        long long fe = 0;
        for (int l = tid; l < k; l += 256) {
            const long long v = cnt[l];
            if (d.problem == kProbMSCP) {
                fe += (long long)(l + 1) * v;
            } else {
                const long long x = v > c1 ? v - c1 : c1 - v;
                const long long y = v > c2 ? v - c2 : c2 - v;
                fe += x < y ? x : y;
            }
        }
        for (int sh = 32; sh >= 1; sh >>= 1) fe += __shfl_xor(fe, sh);
        if ((tid & 63) == 0) fsum[tid >> 6] = fe;
        __syncthreads();
        if (tid == 0) d.feq[m] = fsum[0] + fsum[1] + fsum[2] + fsum[3];
    }
    if (!lists) return;
    {
        // sum_l #V_l^2: the class-mate increments of all rows for this member
        long long q2 = 0;
        for (int l = tid; l < k; l += 256) q2 += (long long)cnt[l] * cnt[l];
        for (int sh = 32; sh >= 1; sh >>= 1) q2 += __shfl_xor(q2, sh);
        if ((tid & 63) == 0) qsum[tid >> 6] = q2;
        __syncthreads();
        if (tid == 0) d.sq[m] = qsum[0] + qsum[1] + qsum[2] + qsum[3];
        if (decide) {
            // the last member block to get here sums every member's value (a ticket
            // counter after a release fence; the last block reads the others' values
            // with atomic loads after an acquire fence) and resets the counter
            int& last_block = *last_block_p;
            if (tid == 0) {
                __threadfence();
                last_block = atomicAdd(&st->prep_ticket, 1) == d.D - 1;
            }
            __syncthreads();
            if (last_block && tid < 64) {
                __threadfence();
                long long w = 0;
                for (int mm = tid; mm < d.D; mm += 64) w += __atomic_load_n(d.sq + mm, __ATOMIC_RELAXED);
                for (int sh = 32; sh >= 1; sh >>= 1) w += __shfl_xor(w, sh);
                if (tid == 0) {
                    st->pdense = penalty_choice(d, w);
                    st->prep_ticket = 0;
                }
            }
        }
    }
    int* offl = cw + NW * k;                        // [k] class starts
    int16_t* lst = (int16_t*)(offl + k);            // [n]
    int32_t* __restrict__ off = d.cls_off + (size_t)m * (k + 1);
    int16_t* __restrict__ cv = d.cls_v + (size_t)m * d.cs;
    // exclusive scan of the counts: runs of `per` classes per thread, the 256 run sums
    // scanned by wave 0 (four per lane, then across lanes)
    const int per = (k + 255) / 256;
    const int lb = min(k, tid * per), le = min(k, lb + per);
    int run = 0;
    for (int l = lb; l < le; ++l) run += cnt[l];
    part[tid] = run;
    __syncthreads();
    if (tid < 64) {
        const int v0 = part[4 * tid], v1 = part[4 * tid + 1], v2 = part[4 * tid + 2], v3 = part[4 * tid + 3];
        const int sum = v0 + v1 + v2 + v3;
        int incl = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o);
            if (tid >= o) incl += y;
        }
        const int ex = incl - sum;
        part[4 * tid] = ex;
        part[4 * tid + 1] = ex + v0;
        part[4 * tid + 2] = ex + v0 + v1;
        part[4 * tid + 3] = ex + v0 + v1 + v2;
    }
    __syncthreads();
    // class l starts at its offset; within it the quarters follow in order, so each
    // wave's cursor for l starts after the earlier quarters' vertices of colour l
    int acc = part[tid];
    for (int l = lb; l < le; ++l) {
        off[l] = acc;
        offl[l] = acc;
        int q = acc;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int x = cw[w * k + l];
            cw[w * k + l] = q;
            q += x;
        }
        acc += cnt[l];
    }
    if (tid == 0) off[k] = n;
    __syncthreads();
    // placement: each vertex takes the next slot of its colour in its wave's range (the
    // order inside a class is not used: the penalty counts do not depend on it), and
    // records its class's start and size for this member
    {
        int* cur = cw + wv * k;
        int2* __restrict__ cinfo = d.cinfo;
        const int qb = wv * Q, qe = min(n, (wv + 1) * Q);
        for (int i0 = qb + lane; i0 < qe; i0 += 64 * kPrepBatch) {
            int xs[kPrepBatch];
#pragma unroll
            for (int u = 0; u < kPrepBatch; ++u) xs[u] = i0 + 64 * u < qe ? (int)gview(c)[i0 + 64 * u] : 0;
#pragma unroll
            for (int u = 0; u < kPrepBatch; ++u) {
                const int i = i0 + 64 * u;
                if (i < qe) {
                    const int x = xs[u];
                    const int pos = atomicAdd(&cur[x], 1);
                    lst[pos] = (int16_t)i;
                    cinfo[(size_t)m * d.cs + i] = make_int2(offl[x], cnt[x]);
                }
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < n; i += 256) cv[i] = lst[i];
}

__global__ __launch_bounds__(256) void k_prep(const GraphDev* __restrict__ gd, int G, int total_mem, int honor_stop,
                                              int next, int decide, int ex_blocks, int advance_prev) {
    const int mem = blockIdx.x;
    if (mem >= total_mem) {
        // blocks past the members: the expansion of the current colours (gate 1), with the
        // same stop decision as the member blocks
        if (mem - total_mem < ex_blocks) expand_block(gd, G, mem - total_mem, honor_stop, next, 1, advance_prev);
        return;
    }
    prep_member(gd, G, mem, honor_stop, next, decide, advance_prev);
}

// -------------------------------------------------------- sparse penalty rows ----

// Penalty rows from the nonzeros of P.  The penalty operand
//   P_ij = t * (a_ij ? 2 alpha lambda x^(alpha-1) : -[i != j or bonus_diag] 2 beta mu x^(beta-1)),
// x = Mt_ij (D - Mt_ij for partitioning), enters the gradient as (P.S_d)[i, l], and
// with one-hot S_d that is the sum of P_ij over the vertices j of colour l in member
// d.  For colouring P_ij vanishes unless j shares row i's colour in some member
// (alpha, beta > 1 give 0^(alpha-1) = 0): a few hundred of the n entries of a row
// in a typical iteration.  One block of NT threads per row i:
//   1. Mt_ij from the class lists: j shares i's colour in member d exactly when j is
//      in the class of c_d(i), so each member adds one to the count of every vertex
//      of that class; the sum_d |class| increments are spread over the whole block.
//      When the classes are large (more than n D / 8 increments: the population
//      briefly collapses into a few giant classes after each smoothing) every j
//      compares its vertex-major colours with row i's instead (n D comparisons);
//   2. the counts become table indices of P_ij, and the nonzero entries go to a list
//      (j, index);
//   3. members are taken PM at a time: every listed j adds P_ij to the accumulator
//      of (d, c_d(j)) for each member d of the group (c_d(j) from the vertex-major
//      colours; consecutive lanes take consecutive members, so the atomics of one
//      instruction hit different accumulators even when a class holds most of the
//      vertices), then the group's sums go to G[d][i][l], added to the contraction's
//      A.S_d (accumulate 1) or written for the contraction's epilogue (accumulate 0).
// A graph choosing per iteration (ps_mode 2) takes these rows only in the iterations
// where the class-size kernel found its classes small; otherwise the contraction's dense pass.
// Steps 1 and 3 issue the loads of their next batch before the atomics of the current
// one.  The sums are taken in 64-bit fixed point: every table value times 2^sc, with sc
// chosen so that n max|P| stays below 2^62, is an integer whenever the table's binary
// exponents span at most 38 - bits(n) (every setting of the paper's parameter grid up
// to n = 4000; beyond, each term is rounded at 2^-sc, at most 2^-30 of max|P| over a
// row), and integer sums do not depend on the order of the additions, so the LDS
// atomics give the same bits on every run.  The result is the sum of the FP32 values
// P_ij, exact in those cases, rounded once to FP32.
// Dynamic LDS (penalty_sparse_lds): table [2 (D + 1) + 1] i64 (the last entry 0, for
// an excluded diagonal), class starts and the prefix of the class sizes [D + 1] i32
// each, the list length, row i's colours [cTs] i16, list [n_pad] u32, then counts
// [n_pad] u32 overlaid by the group's accumulators [PM][k] i64.
// the fitness of one graph (the fitness kernel's body; the fast path runs it in extra
// blocks of the sparse penalty launch, since both follow the contraction)
__device__ __forceinline__ void fitness_graph(const GraphDev* __restrict__ gd, int g, int honor_stop, int flags, int* best);

__host__ __device__ inline size_t ps_tab_words(int D) { return ((size_t)2 * (D + 1) + 1 + 1) & ~(size_t)1; }
__host__ __device__ inline size_t ps_int_words(int D) { return ((size_t)D + 1 + 3) & ~(size_t)3; }
constexpr int kPsBatch = 4;     // entries per thread per batch in steps 1 and 3 (48 registers: eight waves per SIMD)
constexpr int kPsA8 = 2;        // adjacency words per thread loaded at the start

// ---- the row update on the sparse-rows launch (fast path, graphs with pfuse) ----
//
// One wave per (member d, vertex i) row, lane j holding colours j, j + 64, ... (KW of them):
// the added-fitness term, softmax along k (max subtracted), the straight-through gradient
// gW = s^ (gS - sum_l s^_l gS_l), W' = W - eta gW (divided by rho in the smoothing
// iterations) written to the other weight buffer, and the argmax of W' (lowest colour on
// ties) to the other colour buffer.  The arithmetic of the row-update kernel, with the row's
// sums taken over 64 lanes.  The fitness launch that follows accepts the update by flipping
// the buffers, unless the graph stops in this iteration (the stop rule comes before the update).
struct FuseCtx {
    const float* Wc;          // current weights
    float* Wn;                // the other buffer, written
    int16_t* cn;              // the other colour buffer, written
    const int32_t* V;         // class sizes of this iteration (added fitness term)
    float nut, eta, rho;
    bool smooth;
};

__device__ inline FuseCtx fuse_ctx(const GraphDev& d, GraphState* st) {
    FuseCtx f;
    const int pW = st->pW, pS = st->pS;
    const long long t = st->t;
    f.Wc = d.W[pW];
    f.Wn = d.W[pW ^ 1];
    f.cn = d.c[pS ^ 1];
    f.V = d.V[pS];
    f.nut = prob_added(d.problem) ? d.nu * (float)t : 0.0f;
    f.eta = d.eta;
    f.rho = d.rho;
    f.smooth = d.nb_iter > 0 && ((t + 1) % d.nb_iter) == 0;
    return f;
}

// loads of row (dd, i): weights and the raw G entries (fp32 bits, or the uint16 A.S count) of
// the lane's colours below k; one base address per row, so the loads take immediate offsets
template <int KW>
__device__ inline void fuse_row_load(const GraphDev& d, const FuseCtx& f, int dd, int i, int lane, bool g16,
                                     float (&wv)[KW], uint32_t (&gr)[KW]) {
    const int k = d.k;
    const size_t row = ((size_t)dd * d.n + i) * k + lane;
    const auto* __restrict__ w = gview(f.Wc) + row;
    const auto* __restrict__ g32 = gview((const float*)d.G) + row;
    const auto* __restrict__ g16p = gview((const uint16_t*)d.G) + row;
#pragma unroll
    for (int q = 0; q < KW; ++q) {
        wv[q] = 0.0f;
        gr[q] = 0u;
        if (lane + 64 * q < k) {
            wv[q] = w[64 * q];
            gr[q] = g16 ? (uint32_t)g16p[64 * q] : __float_as_uint(g32[64 * q]);
        }
    }
}

// gv: the lane's entries of gS without the added-fitness term (entries past k are ignored)
template <int KW, int ADD>
__device__ inline void fuse_row_update(const GraphDev& d, GraphState* st, const FuseCtx& f, int dd, int i, int lane,
                                       const float (&wv)[KW], float (&gv)[KW]) {
    const int k = d.k;
    if (ADD && f.nut != 0.0f) {
        const auto* __restrict__ V = gview(f.V) + (size_t)dd * k + lane;
#pragma unroll
        for (int q = 0; q < KW; ++q)
            if (lane + 64 * q < k) gv[q] += f.nut * added_grad(d.problem, V[64 * q], lane + 64 * q, d.c1, d.c2);
    }
    float mx = -INFINITY;
#pragma unroll
    for (int q = 0; q < KW; ++q)
        if (lane + 64 * q < k) mx = fmaxf(mx, wv[q]);
    mx = wave_max(mx);
    float e[KW];
    float z = 0.0f, qs = 0.0f;
#pragma unroll
    for (int q = 0; q < KW; ++q) {
        e[q] = (lane + 64 * q < k) ? exp_soft(wv[q] - mx) : 0.0f;
        z += e[q];
        qs += e[q] * gv[q];
    }
    z = wave_sum(z);
    qs = wave_sum(qs);
    const float rz = 1.0f / z;
    const float rq = qs * rz;
    float* __restrict__ wo = f.Wn + ((size_t)dd * d.n + i) * k + lane;
    float best = -INFINITY;
    int bi = 0x7FFFFFFF;
    bool bad = false;
#pragma unroll
    for (int q = 0; q < KW; ++q) {
        const int l = lane + 64 * q;
        if (l < k) {
            const float step = e[q] * rz * (gv[q] - rq);
            float nw = wv[q] - f.eta * step;
            if (f.smooth) nw = nw / f.rho;
            wo[64 * q] = nw;
            if (!finite_f(nw)) bad = true;
            if (nw > best) { best = nw; bi = l; }
        }
    }
    // the argmax: the largest value, then the lowest colour holding it
    const int bo = f32_ord(best);
    const int bmax = wave_max_i(bo);
    const int arg = wave_min_i(bo == bmax ? bi : 0x7FFFFFFF);
    const bool any_bad = __any(bad);
    if (lane == 0) {
        int c = arg;
        if (any_bad || c >= k) {
            c = 0;
            atomicExch(&st->next_bad, 1);
        }
        f.cn[(size_t)dd * d.cs + i] = (int16_t)c;
    }
}

// the row update alone for every member of vertex i (iterations of a pfuse graph whose penalty
// took the dense pass, or without a penalty): G holds the whole fp32 gradient; each wave takes
// members wave, wave + NT/64, ... (the launch's blocks per CU keep enough rows in flight)
template <int NT, int KW, int ADD>
__device__ __forceinline__ void fuse_update_only(const GraphDev& d, GraphState* st, int i) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const FuseCtx f = fuse_ctx(d, st);
    for (int dd = wave; dd < d.D; dd += NW) {
        float wv[KW], gv[KW];
        uint32_t gr[KW];
        fuse_row_load<KW>(d, f, dd, i, lane, false, wv, gr);
#pragma unroll
        for (int q = 0; q < KW; ++q) gv[q] = __uint_as_float(gr[q]);
        fuse_row_update<KW, ADD>(d, st, f, dd, i, lane, wv, gv);
    }
}

// The fused variants with at most five values per lane are held to 64 registers (eight waves per
// SIMD): with their 35 KB of LDS at n = 4000, k = 280, D = 32 that runs four 512-thread blocks per
// CU instead of three (the step 0.321 -> 0.310 ms there; two registers spill in the variant with
// an added fitness term).
template <int NT, int KW, int ADD>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT == 512 && KW > 0 && KW <= 5 ? 8 : 1))) void
k_pen_sparse(const GraphDev* __restrict__ gd, int G, int total_blocks, int honor_stop, int PM, int accumulate) {
    extern __shared__ __attribute__((aligned(16))) uint8_t ps_sh[];
    constexpr int B = KW > 0 ? 2 : kPsBatch;
    const int b = blockIdx.x;
    if (b >= total_blocks) return;
    const GraphDev& d = gd[find_graph(gd, G, b, [](const GraphDev& x) { return x.ps_begin; })];
    GraphState* st = d.st;
    if (honor_stop && st->stopped) return;
    const bool sparse_now = d.psparse && !st->pdense && pen_active(d, st);
    // graphs whose row update rides on this launch (the fast path's sparse graphs)
    const bool fuse = KW > 0 && d.pfuse && accumulate;
    if constexpr (KW > 0) {
        if (fuse && !sparse_now) {
            fuse_update_only<NT, KW, ADD>(d, st, b - d.ps_begin);
            return;
        }
    }
    if (!sparse_now) return;
    const int n = d.n, k = d.k, D = d.D, cs = d.cs;
    const int n_pad = d.n_pad;
    const size_t cTs = d.cTs;
    const int i = b - d.ps_begin;
    const int tid = threadIdx.x, lane = tid & 63;
    const int T = 2 * (D + 1) + 1, zslot = T - 1;
    long long* tab = (long long*)ps_sh;                       // [ps_tab_words(D)]
    int* cbeg = (int*)(tab + ps_tab_words(D));                 // [ps_int_words(D)]
    int* pre = cbeg + ps_int_words(D);                         // [ps_int_words(D)]
    int* nzc = pre + ps_int_words(D);                          // [4]: list length, max-exponent
    int16_t* ci = (int16_t*)(nzc + 4);                         // [cTs]
    uint32_t* list = (uint32_t*)(ci + cTs);                    // [n_pad]
    uint32_t* cnt = list + n_pad;                              // [n_pad], steps 1-2
    unsigned long long* acc = (unsigned long long*)cnt;        // [PM][k], step 3
    const float tf = (float)st->t;
    const bool diag = d.bonus_diag != 0;
    const int16_t* __restrict__ cT = d.cT;
    // partitioning: the values are those of the dense operand, whose product the
    // contraction negates along with A.S
    const float sgn = prob_partition(d.problem) ? -1.0f : 1.0f;

    // 0. the adjacency bytes of step 2's first passes, the row's colours and classes,
    // the value table (one round of loads); counts cleared; the table's largest magnitude
    constexpr int TV = (2 * (kMaxD + 1) + 1 + NT - 1) / NT;   // table entries per thread
    float tv[TV];
#pragma unroll
    for (int u = 0; u < TV; ++u) {
        const int vi = tid + u * NT;
        tv[u] = 0.0f;
        if (vi < T - 1) tv[u] = vi <= D ? -(tf * gview(d.lut_bon)[vi]) : tf * gview(d.lut_pen)[vi - D - 1];
    }
    const uint8_t* __restrict__ arow = d.A8 + (size_t)i * n_pad;
    uint32_t a4pre[kPsA8];
#pragma unroll
    for (int u = 0; u < kPsA8; ++u) {
        const int j0 = 4 * (tid + u * NT);
        a4pre[u] = j0 < n ? gview((const uint32_t*)(arow + j0))[0] : 0u;
    }
    for (int dm = tid; dm < (int)cTs; dm += NT) {
        ci[dm] = gview(cT)[(size_t)i * cTs + dm];
        if (dm < D) {
            // (start, size) as one 8-byte load: start in the low word
            const unsigned long long cl = gview((const unsigned long long*)d.cinfo)[(size_t)dm * d.cs + i];
            cbeg[dm] = (int)(uint32_t)cl;
            pre[dm + 1] = (int)(uint32_t)(cl >> 32);
        }
    }
    for (int e = tid; e < n_pad / 4; e += NT) ((u32x4n*)cnt)[e] = u32x4n{0u, 0u, 0u, 0u};
    if (tid == 0) { nzc[0] = 0; nzc[1] = 0; pre[0] = 0; }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < TV; ++u) {
        if (tv[u] != 0.0f) {
            int ex;
            frexpf(tv[u], &ex);
            // exponents are compared as ex + 256 > 0 (the counter starts at 0 = none)
            atomicMax(&nzc[1], ex + 256);
        }
    }
    // prefix of the class sizes (wave 0, 64 members at a time)
    if (tid < 64) {
        int carry = 0;
        for (int base = 0; base < D; base += 64) {
            const int dm = base + lane;
            int x = dm < D ? pre[dm + 1] : 0;
#pragma unroll
            for (int sh = 1; sh < 64; sh <<= 1) {
                const int y = __shfl_up(x, sh);
                if (lane >= sh) x += y;
            }
            if (dm < D) pre[dm + 1] = carry + x;
            carry += __shfl(x, 63);
        }
    }
    __syncthreads();
    // fixed-point scale: |P_ij| < 2^E1 and n < 2^E2, so sums stay below 2^(E1 + E2) <= 2^62
    const int emax = nzc[1];
    const int sc = 62 - ((emax > 0 ? emax - 256 : 0) + (32 - __builtin_clz((unsigned)n)));
#pragma unroll
    for (int u = 0; u < TV; ++u) {
        const int vi = tid + u * NT;
        if (vi < T) tab[vi] = (long long)rint(ldexp((double)tv[u], sc));
    }
    // 1. Mt_ij
    const int W1 = pre[D];
    if ((long long)W1 * 8 <= (long long)n * D) {
        // from the class lists: entry q of the concatenated classes belongs to member dm
        // with pre[dm] <= q < pre[dm + 1] (found once by bisection, then advanced)
        int dm = 0;
        if (tid < W1) {
            int lo = 0, hi = D - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (pre[mid] <= tid) lo = mid; else hi = mid - 1;
            }
            dm = lo;
        }
        int js[B];
        auto fetch = [&](int q0) {
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int q = q0 + u * NT;
                js[u] = -1;
                if (q < W1) {
                    while (pre[dm + 1] <= q) ++dm;
                    js[u] = gview(d.cls_v)[(size_t)dm * cs + cbeg[dm] + (q - pre[dm])];
                }
            }
        };
        fetch(tid);
        for (int q0 = tid; q0 < W1; q0 += B * NT) {
            int cur[B];
#pragma unroll
            for (int u = 0; u < B; ++u) cur[u] = js[u];
            if (q0 + B * NT < W1) fetch(q0 + B * NT);
#pragma unroll
            for (int u = 0; u < B; ++u)
                if (cur[u] >= 0) atomicAdd(&cnt[cur[u]], 1u);
        }
    } else {
        // by comparison: eight members per 16-byte word of a vertex-major row; members
        // beyond D (the row padding) are masked out
        const int nw = (int)(cTs / 8);
        for (int j0 = tid; j0 < n; j0 += 2 * NT) {
            int m2[2] = {0, 0};
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int j = j0 + u * NT;
                if (j >= n) continue;
                const int16_t* row = cT + (size_t)j * cTs;
                for (int w = 0; w < nw; ++w) {
                    const u32x4n x = gload16(row + 8 * w);
                    const u32x4n y = *(const u32x4n*)(ci + 8 * w);
                    const uint32_t xs[4] = {x.x, x.y, x.z, x.w}, ys[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
                    for (int h = 0; h < 4; ++h) {
                        const int m0 = 8 * w + 2 * h;
                        const uint32_t valid = (m0 < D ? 0x8000u : 0u) | (m0 + 1 < D ? 0x80000000u : 0u);
                        m2[u] += equal_halves_in(xs[h], ys[h], valid);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < 2; ++u)
                if (j0 + u * NT < n) cnt[j0 + u * NT] = (uint32_t)m2[u];
        }
    }
    __syncthreads();
    // 2. table index of P_ij for every j; the nonzero entries go to the list
    for (int base = 0, pass = 0; base < n; base += 4 * NT, ++pass) {
        const int j0 = base + 4 * tid;
        int vi[4];
        bool nz[4];
        if (j0 < n) {
            uint32_t a4 = 0;
            if (pass < kPsA8) {
#pragma unroll
                for (int u = 0; u < kPsA8; ++u)
                    if (u == pass) a4 = a4pre[u];
            } else {
                a4 = gview((const uint32_t*)(arow + j0))[0];
            }
            const u32x4n c4 = *(const u32x4n*)(cnt + j0);
            const uint32_t cw[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = j0 + u;
                const bool edge = ((a4 >> (8 * u)) & 0xFFu) != 0;
                const bool excl = !edge && !diag && j == i;
                vi[u] = excl ? zslot : (edge ? D + 1 + (int)cw[u] : (int)cw[u]);
                nz[u] = j < n && tab[vi[u]] != 0;
            }
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) { vi[u] = zslot; nz[u] = false; }
        }
        unsigned long long bal[4];
        int tot = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            bal[u] = __ballot(nz[u]);
            tot += __popcll(bal[u]);
        }
        int off = 0;
        if (lane == 0 && tot > 0) off = atomicAdd(&nzc[0], tot);
        off = __shfl(off, 0);
        const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (nz[u]) list[off + __popcll(bal[u] & below)] = (uint32_t)(j0 + u) | ((uint32_t)vi[u] << 16);
            off += __popcll(bal[u]);
        }
    }
    __syncthreads();
    const int nnz = nzc[0];
    // 3. members PM (= 8) at a time
    __attribute__((address_space(1))) float* Gg = (__attribute__((address_space(1))) float*)d.G;
    const double inv = ldexp(1.0, -sc);
    constexpr int KWF = KW > 0 ? KW : 1;
    FuseCtx fc{};
    if constexpr (KW > 0)
        if (fuse) fc = fuse_ctx(d, st);
    const int wave = tid >> 6;
    for (int d0 = 0; d0 < D; d0 += PM) {
        const int pm = min(PM, D - d0);
        // fused: wave w < pm loads row (d0 + w, i) of the weights and of the uint16 A.S counts
        // now, behind the accumulation below (PM is at most the block's wave count)
        float wv[KWF];
        uint32_t gr[KWF];
        if constexpr (KW > 0)
            if (fuse && wave < pm) fuse_row_load<KW>(d, fc, d0 + wave, i, lane, true, wv, gr);
        // f_color (fast path): thread dd < pm loads the contraction's (A.S)[i, c_d(i)] of member
        // d0 + dd now, behind the accumulation below, and adds it to the slots before the barrier
        // that precedes this group's read-modify-write of G (or its row updates)
        float own = 0.0f;
        if (accumulate && tid < pm) {
            const size_t o = ((size_t)(d0 + tid) * n + i) * k + ci[d0 + tid];
            own = fuse ? (float)gview((const uint16_t*)d.G)[o] : sgn * Gg[o];
        }
        // the accumulators start at zero: cleared here before the first group (they share their
        // words with the counts of steps 1-2), and by the fused row updates, which clear each
        // member's row once they have read it, before the later groups
        if (!fuse || d0 == 0) {
            for (int e = tid; e < pm * k / 2; e += NT) ((u32x4n*)acc)[e] = u32x4n{0u, 0u, 0u, 0u};
            if ((pm * k) & 1)
                if (tid == 0) acc[pm * k - 1] = 0ull;
            __syncthreads();
        }
        // one list entry per thread: the colours of its vertex j in the group's (at most eight)
        // members come in one 16-byte word of the vertex-major colours (rows padded to a multiple
        // of eight), and each member's accumulator of that colour takes P_ij.  The next entry's
        // word is loaded before this entry's LDS atomics.
        const auto* __restrict__ cTg = gview(cT);
        auto word = [&](int e, u32x4n& w, int& vi) {
            vi = 0;
            if (e < nnz) {
                const uint32_t ent = list[e];
                w = *(const __attribute__((address_space(1))) u32x4n*)(cTg + (size_t)(ent & 0xFFFFu) * cTs + d0);
                vi = (int)(ent >> 16);
            }
        };
        u32x4n wn = {0u, 0u, 0u, 0u};
        int vn;
        word(tid, wn, vn);
        for (int e = tid; e < nnz; e += NT) {
            const u32x4n wc = wn;
            const int vc = vn;
            word(e + NT, wn, vn);
            const unsigned long long v = (unsigned long long)tab[vc];
#pragma unroll
            for (int h = 0; h < 8; ++h) {
                if (h < pm) {
                    const int c = (int)((wc[h >> 1] >> (16 * (h & 1))) & 0xFFFFu);
                    atomicAdd(&acc[h * k + c], v);
                }
            }
        }
        // the number of row i's neighbours sharing its colour (the gather of 2 f_color)
        if (accumulate && tid < pm)
            atomicAdd(&d.f2p[(size_t)(d0 + tid) * kF2Slots + (i & (kF2Slots - 1))], (int)own);
        __syncthreads();
        if constexpr (KW > 0) {
            if (fuse) {
                // gS = sgn (A.S + P.S) for row (d0 + wave, i): the member's sums to FP32 (sgn P.S)
                // and added to the A.S counts, rounded as the unfused path rounds the stored G;
                // the row's accumulators are cleared for the next group; then the row update
                if (wave < pm) {
                    float gv[KW];
                    unsigned long long* __restrict__ ar = acc + wave * k + lane;
#pragma unroll
                    for (int q = 0; q < KW; ++q) {
                        gv[q] = 0.0f;
                        if (lane + 64 * q < k) {
                            gv[q] = sgn * (float)gr[q] + sgn * (float)((double)(long long)ar[64 * q] * inv);
                            ar[64 * q] = 0ull;
                        }
                    }
                    fuse_row_update<KW, ADD>(d, st, fc, d0 + wave, i, lane, wv, gv);
                }
                __syncthreads();
                continue;
            }
        }
        for (int e0 = tid; e0 < pm * k; e0 += 4 * NT) {
            float prev[4];
            size_t off[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * NT;
                prev[u] = 0.0f;
                off[u] = 0;
                if (e < pm * k) {
                    const int dd = e / k, l = e - dd * k;
                    off[u] = ((size_t)(d0 + dd) * n + i) * k + l;
                    if (accumulate) prev[u] = Gg[off[u]];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * NT;
                if (e < pm * k) Gg[off[u]] = prev[u] + sgn * (float)((double)(long long)acc[e] * inv);
            }
        }
        __syncthreads();
    }
}


// One-hot S^T [rows (d,l)][cols j] in the operand format; 16 columns per thread
// (fp4: two columns per byte, the lower in the low nibble, 1.0 = 0x2).  For FP8
// graphs the bf16 copy used by the penalty pass is written as well (the fp4 penalty
// pass reads the fp4 operand itself).
__device__ __forceinline__ void expand_block(const GraphDev* __restrict__ gd, int G, int b, int honor_stop, int next, int gate,
                             int adv) {
    const GraphDev& d = gd[find_graph(gd, G, b, [](const GraphDev& x) { return x.ex_begin; })];
    GraphState* st = d.st;
    if (honor_stop && (st->stopped || (adv && st->next_bad))) return;
    const int p = next ? st->pS ^ 1 : st->pS;
    // the bf16 copy of S feeds only the dense penalty pass of FP8 graphs
    const bool want_sp2 = prec_split(d.precision) && (!gate || !d.psparse || st->pdense);
    // a thread takes 16 columns of kExpandRows consecutive colour rows of one member: their
    // colours are loaded once for all of its rows
    const int cgs = d.n_pad / 16;
    const int kr = (d.k + kExpandRows - 1) / kExpandRows;   // row groups per member
    const long long item = (long long)(b - d.ex_begin) * 256 + threadIdx.x;
    const long long rg = item / cgs;
    const int cg = (int)(item - rg * cgs);
    if (rg >= (long long)d.D * kr) return;
    const int dm = (int)(rg / kr);
    const int l0 = (int)(rg - (long long)dm * kr) * kExpandRows;
    const int j0 = cg * 16;
    const int CM = d.cmax;
    uint32_t w1[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};   // the member's 16 colours (one colour per vertex)
    if (CM == 1 && j0 < d.n) {
        // 16 colours in two 16-byte loads (rows are padded to 64 entries)
        const int16_t* c = d.c[p] + (size_t)dm * d.cs;
        const uint4 a = *(const uint4*)(c + j0);
        const uint4 bb = *(const uint4*)(c + j0 + 8);
        w1[0] = a.x; w1[1] = a.y; w1[2] = a.z; w1[3] = a.w;
        w1[4] = bb.x; w1[5] = bb.y; w1[6] = bb.z; w1[7] = bb.w;
    }
#pragma unroll 1
    for (int rr = 0; rr < kExpandRows; ++rr) {
    const int l = l0 + rr;
    if (l >= d.k) break;
    const int row = dm * d.k + l;
    uint32_t mask = 0;   // bit q set when column j0+q has colour l (one of its colours: multicolouring)
    if (j0 < d.n) {
        if (CM == 1) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int col = (int)((w1[q >> 1] >> (16 * (q & 1))) & 0xFFFFu);
                if (j0 + q < d.n && col == l) mask |= 1u << q;
            }
        } else {
            for (int sl = 0; sl < CM; ++sl) {
                const int16_t* c = d.sel + ((size_t)dm * CM + sl) * d.cs;
                const uint4 a = *(const uint4*)(c + j0);
                const uint4 bb = *(const uint4*)(c + j0 + 8);
                const uint32_t w[8] = {a.x, a.y, a.z, a.w, bb.x, bb.y, bb.z, bb.w};
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int col = (int)((w[q >> 1] >> (16 * (q & 1))) & 0xFFFFu);
                    if (j0 + q < d.n && col == l) mask |= 1u << q;
                }
            }
        }
    }
    const size_t off = (size_t)row * d.n_pad + j0;
    if (d.precision == kPrecFP32) {
        float4* o = (float4*)((float*)d.Sop[p] + off);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float4 x;
            x.x = (mask >> (4 * v + 0)) & 1 ? 1.0f : 0.0f;
            x.y = (mask >> (4 * v + 1)) & 1 ? 1.0f : 0.0f;
            x.z = (mask >> (4 * v + 2)) & 1 ? 1.0f : 0.0f;
            x.w = (mask >> (4 * v + 3)) & 1 ? 1.0f : 0.0f;
            o[v] = x;
        }
    } else {
        // bf16: the BF16 operand itself, or the FP8 graphs' copy for the penalty pass
        const bool bf16_out = d.precision == kPrecBF16 || want_sp2;
        uint16_t* sb = d.precision == kPrecBF16 ? (uint16_t*)d.Sop[p] : (uint16_t*)d.Sp2[p];
        uint4* o = (uint4*)(sb + off);
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            if (!bf16_out) break;
            uint32_t w[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                int q = 8 * v + 2 * h;
                w[h] = (((mask >> q) & 1) ? 0x3F80u : 0u) | (((mask >> (q + 1)) & 1) ? 0x3F800000u : 0u);
            }
            o[v] = make_uint4(w[0], w[1], w[2], w[3]);
        }
        if (d.precision == kPrecFP8) {
            uint32_t w[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                uint32_t x = 0;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if ((mask >> (4 * h + e)) & 1) x |= 0x38u << (8 * e);
                w[h] = x;
            }
            *(uint4*)((uint8_t*)d.Sop[p] + off) = make_uint4(w[0], w[1], w[2], w[3]);
        } else if (d.precision == kPrecFP4) {
            uint32_t w[2] = {0u, 0u};
#pragma unroll
            for (int q = 0; q < 16; ++q)
                if ((mask >> q) & 1) w[q >> 3] |= 0x2u << (4 * (q & 7));
            *(uint2*)((uint8_t*)d.Sop[p] + (off >> 1)) = make_uint2(w[0], w[1]);
        }
    }
    }
}

__global__ __launch_bounds__(256) void k_expand(const GraphDev* __restrict__ gd, int G, int total_blocks,
                                                int honor_stop, int next, int gate) {
    const int b = blockIdx.x;
    if (b >= total_blocks) return;
    expand_block(gd, G, b, honor_stop, next, gate, 0);
}

// ------------------------------------------------------------ step 3 -----------

// Group concentration Mt_ij = #{d : c_d(i) = c_d(j)} over TS x TS tiles of the
// upper triangle (mirrored; TS = 64, or 32 when n_pad <= 2048 so small graphs still
// give every CU work), and from it the penalty operand
//   P_ij = t * (a_ij ? 2 alpha lambda m^(alpha-1) : -[i != j or bonus_diag] 2 beta mu m^(beta-1)).
// Optional: Mt to mt_out (int32 [n][n]) and kappa / varpi partial sums.  Each of the
// 256 threads owns a PT x PT block of the tile (PT = TS / 16).
constexpr int kMtChunk = 128;   // members per LDS chunk

template <int PT>
__device__ __forceinline__ void mtilde_tile(const GraphDev& d, GraphState* st, int b, int flags, int32_t* __restrict__ mt_out,
                            int16_t (*ci)[64], int16_t (*cj)[64], double (*red)[256]) {
    constexpr int TS = 16 * PT;
    const float tf = (float)st->t;
    const bool pen = (d.lambda * tf != 0.0f) || (d.mu * tf != 0.0f);
    const int p = st->pS;
    // upper-triangle tile (ti <= tj)
    int u = b - d.mt_begin, ti = 0, T = d.mt_T;
    while (u >= T - ti) { u -= T - ti; ++ti; }
    const int tj = ti + u;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i0 = ti * TS, j0 = tj * TS;
    int cnt[PT][PT];
#pragma unroll
    for (int a = 0; a < PT; ++a)
#pragma unroll
        for (int q = 0; q < PT; ++q) cnt[a][q] = 0;
    // rows of colours: members (one colour per vertex), or for multicolouring (member, slot)
    // pairs of the selection, whose slots of a member must meet in one chunk
    const int CM = d.cmax;
    const int16_t* base = CM > 1 ? d.sel : d.c[p];
    const int vrows = d.D * CM;
    const int chunk = (kMtChunk / CM) * CM;
    for (int dbase = 0; dbase < vrows; dbase += chunk) {
        const int dn = min(chunk, vrows - dbase);
        __syncthreads();
        for (int e = threadIdx.x; e < dn * TS; e += 256) {
            const int dm = e / TS, x = e - dm * TS;
            const int16_t* cr = base + (size_t)(dbase + dm) * d.cs;
            // out-of-range vertices and unselected slots get distinct sentinels so they never match
            const int16_t a = (i0 + x < d.n) ? cr[i0 + x] : (int16_t)-1;
            const int16_t b = (j0 + x < d.n) ? cr[j0 + x] : (int16_t)-2;
            ci[dm][x] = a < 0 ? (int16_t)-1 : a;
            cj[dm][x] = b < 0 ? (int16_t)-2 : b;
        }
        __syncthreads();
        if (CM == 1) {
            for (int dm = 0; dm < dn; ++dm) {
                int16_t av[PT], bv[PT];
#pragma unroll
                for (int a = 0; a < PT; ++a) {
                    av[a] = ci[dm][ty * PT + a];
                    bv[a] = cj[dm][tx * PT + a];
                }
#pragma unroll
                for (int a = 0; a < PT; ++a)
#pragma unroll
                    for (int q = 0; q < PT; ++q) cnt[a][q] += (av[a] == bv[q]) ? 1 : 0;
            }
        } else {
            // the colours i and j share within each member: every slot against every slot
            for (int mm = 0; mm < dn; mm += CM)
                for (int s1 = 0; s1 < CM; ++s1) {
                    int16_t av[PT];
#pragma unroll
                    for (int a = 0; a < PT; ++a) av[a] = ci[mm + s1][ty * PT + a];
                    for (int s2 = 0; s2 < CM; ++s2) {
                        int16_t bv[PT];
#pragma unroll
                        for (int q = 0; q < PT; ++q) bv[q] = cj[mm + s2][tx * PT + q];
#pragma unroll
                        for (int a = 0; a < PT; ++a)
#pragma unroll
                            for (int q = 0; q < PT; ++q) cnt[a][q] += (av[a] == bv[q]) ? 1 : 0;
                    }
                }
        }
    }
    const bool mirror = ti != tj;
    double ka = 0.0, vb = 0.0;
    const bool fp32 = d.precision == kPrecFP32;
    // fields used between the stores below stay in registers (no reload through gd)
    const int n = d.n;
    const size_t n_pad = d.n_pad;
    const uint8_t* __restrict__ A8 = d.A8;
    const float* __restrict__ lut_pen = d.lut_pen;
    const float* __restrict__ lut_bon = d.lut_bon;
    const double* __restrict__ lut_ka = d.lut_ka;
    const double* __restrict__ lut_vb = d.lut_vb;
    const bool bdiag = d.bonus_diag != 0;
    void* __restrict__ Pop = d.Pop;
    // the thread's block: rows i0 + PT ty + a, columns j0 + PT tx + q; the adjacency of a
    // row's PT columns is one load (A8 rows are n_pad bytes, PT | j), and the operand goes
    // out as one vector store per row of the block and per row of its mirror
    const int ib = i0 + ty * PT, jb = j0 + tx * PT;
    float val[PT][PT];
#pragma unroll
    for (int a = 0; a < PT; ++a) {
        const int i = ib + a;
        uint32_t arow;
        if constexpr (PT == 4)
            arow = gview((const uint32_t*)(A8 + (size_t)i * n_pad + jb))[0];
        else
            arow = gview((const uint16_t*)(A8 + (size_t)i * n_pad + jb))[0];
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            const int j = jb + q;
            float v = 0.0f;
            if (i < n && j < n) {
                const int m = cnt[a][q];
                const bool edge = ((arow >> (8 * q)) & 0xFFu) != 0;
                const bool bon = !edge && (i != j || bdiag);
                if (edge) v = tf * lut_pen[m];
                else if (bon) v = -(tf * lut_bon[m]);
                if (flags & kFlagLoss) {
                    const double wgt = mirror ? 2.0 : 1.0;
                    if (edge) ka += wgt * lut_ka[m];
                    else if (bon) vb += wgt * lut_vb[m];
                }
                if ((flags & kFlagMtOut) && mt_out) {
                    mt_out[(size_t)i * n + j] = m;
                    if (mirror) mt_out[(size_t)j * n + i] = m;
                }
            }
            val[a][q] = v;
        }
    }
    if (pen || (flags & kFlagForcePen)) {
        if (fp32) {
#pragma unroll
            for (int a = 0; a < PT; ++a) {
                float* o = (float*)Pop + (size_t)(ib + a) * n_pad + jb;
                if constexpr (PT == 4) *(float4*)o = make_float4(val[a][0], val[a][1], val[a][2], val[a][3]);
                else *(float2*)o = make_float2(val[a][0], val[a][1]);
            }
            if (mirror) {
#pragma unroll
                for (int q = 0; q < PT; ++q) {
                    float* o = (float*)Pop + (size_t)(jb + q) * n_pad + ib;
                    if constexpr (PT == 4) *(float4*)o = make_float4(val[0][q], val[1][q], val[2][q], val[3][q]);
                    else *(float2*)o = make_float2(val[0][q], val[1][q]);
                }
            }
        } else {
            // fp4 graphs: the penalty pass multiplies by 2 S (cheaper to widen from fp4), so
            // their operand is stored halved, exactly
            if (d.precision == kPrecFP4) {
#pragma unroll
                for (int a = 0; a < PT; ++a)
#pragma unroll
                    for (int q = 0; q < PT; ++q) val[a][q] *= 0.5f;
            }
#pragma unroll
            for (int a = 0; a < PT; ++a) {
                uint16_t* o = (uint16_t*)Pop + (size_t)(ib + a) * n_pad + jb;
                const uint32_t lo = f32_to_bf16_rne(val[a][0]) | ((uint32_t)f32_to_bf16_rne(val[a][1]) << 16);
                if constexpr (PT == 4) {
                    const uint32_t hi = f32_to_bf16_rne(val[a][2]) | ((uint32_t)f32_to_bf16_rne(val[a][3]) << 16);
                    *(uint2*)o = make_uint2(lo, hi);
                } else {
                    *(uint32_t*)o = lo;
                }
            }
            if (mirror) {
#pragma unroll
                for (int q = 0; q < PT; ++q) {
                    uint16_t* o = (uint16_t*)Pop + (size_t)(jb + q) * n_pad + ib;
                    const uint32_t lo = f32_to_bf16_rne(val[0][q]) | ((uint32_t)f32_to_bf16_rne(val[1][q]) << 16);
                    if constexpr (PT == 4) {
                        const uint32_t hi = f32_to_bf16_rne(val[2][q]) | ((uint32_t)f32_to_bf16_rne(val[3][q]) << 16);
                        *(uint2*)o = make_uint2(lo, hi);
                    } else {
                        *(uint32_t*)o = lo;
                    }
                }
            }
        }
    }
    if (flags & kFlagLoss) {
        red[0][threadIdx.x] = ka;
        red[1][threadIdx.x] = vb;
        __syncthreads();
        for (int s = 128; s >= 1; s >>= 1) {
            if (threadIdx.x < s) {
                red[0][threadIdx.x] += red[0][threadIdx.x + s];
                red[1][threadIdx.x] += red[1][threadIdx.x + s];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            d.part[2 * (b - d.mt_begin) + 0] = red[0][0];
            d.part[2 * (b - d.mt_begin) + 1] = red[1][0];
        }
    }
}

// tile b (flattened over the graphs) of the group-concentration kernel; ci, cj, red: its LDS
__device__ __forceinline__ void mtilde_block(const GraphDev* __restrict__ gd, int G, int b, int honor_stop, int flags, int gsel,
                             int32_t* __restrict__ mt_out, int16_t (*ci)[64], int16_t (*cj)[64], double (*red)[256]) {
    const int g = find_graph(gd, G, b, [](const GraphDev& x) { return x.mt_begin; });
    const GraphDev& d = gd[g];
    GraphState* st = d.st;
    if (honor_stop && st->stopped) return;
    if (gsel >= 0 && g != gsel) return;
    const float tf = (float)st->t;
    const bool pen = (d.lambda * tf != 0.0f) || (d.mu * tf != 0.0f);
    if (!pen && !(flags & (kFlagForcePen | kFlagLoss | kFlagMtOut))) return;
    if ((flags & kFlagGate) && d.psparse && !st->pdense) return;
    if (d.mt_ts == 32)
        mtilde_tile<2>(d, st, b, flags, mt_out, ci, cj, red);
    else
        mtilde_tile<4>(d, st, b, flags, mt_out, ci, cj, red);
}
__global__ __launch_bounds__(256) void k_mtilde(const GraphDev* __restrict__ gd, int G, int total_tiles,
                                                int honor_stop, int flags, int gsel, int32_t* __restrict__ mt_out) {
    __shared__ int16_t ci[kMtChunk][64];
    __shared__ int16_t cj[kMtChunk][64];
    __shared__ double red[2][256];
    const int b = blockIdx.x;
    if (b >= total_tiles) return;
    mtilde_block(gd, G, b, honor_stop, flags, gsel, mt_out, ci, cj, red);
}

// ------------------------------------------------------- step 2, stop rule -----

// One block per graph: f_color = f2 / 2 (f2 gathered from A.S); the main
// fitness f_color, or |E| - f_color for partitioning; the added fitness (f_eq, or
// the colour cost sum_l (l + 1) #V_l) as the class-size kernel left it; f = main + added;
// lowest legal member; stop rule.  Clears f2.  With kFlagReport only the fitness
// arrays are written.
__device__ __forceinline__ void fitness_graph(const GraphDev* __restrict__ gd, int g, int honor_stop, int flags, int* best_sh) {
    int& best = *best_sh;
    const GraphDev& d = gd[g];
    GraphState* st = d.st;
    if (honor_stop && st->stopped) return;
    const bool sparse_now = d.psparse && !st->pdense && pen_active(d, st);
    const int p = st->pS;
    if (threadIdx.x == 0) best = 0x7FFFFFFF;
    if ((flags & kFlagFoldSparse) && sparse_now) {
        // this iteration's sparse rows gathered 2 f_color into slots: fold and clear them
        for (int m = threadIdx.x; m < d.D; m += blockDim.x) {
            int sum = 0;
            for (int sl = 0; sl < kF2Slots; ++sl) {
                sum += d.f2p[(size_t)m * kF2Slots + sl];
                d.f2p[(size_t)m * kF2Slots + sl] = 0;
            }
            d.f2[m] = sum;
        }
    }
    __syncthreads();
    // the added fitness (equity or colour cost) was reduced by the class-size kernel
    const bool added = prob_added(d.problem);
    for (int m = threadIdx.x; m < d.D; m += blockDim.x) {
        long long fc = d.f2[m] / 2;
        if (prob_partition(d.problem)) fc = (d.ones_dev ? (long long)(*d.ones_dev / 2) : d.edges) - fc;
        const long long fe = added ? d.feq[m] : 0;
        d.fcol[m] = fc;
        d.feq[m] = fe;
        d.f[m] = fc + fe;
        d.f2[m] = 0;
        if (fc + fe == 0) atomicMin(&best, m);
    }
    __syncthreads();
    if (flags & kFlagReport) return;
    if (threadIdx.x == 0) {
        // the route this iteration's penalty product took (the contraction and the sparse
        // rows read the same state)
        if (!pen_active(d, st)) st->it_nopen += 1;
        else if ((flags & kFlagPlainPen) || !d.psparse || st->pdense) st->it_dense += 1;
        else st->it_sparse += 1;
    }
    const int ld = best == 0x7FFFFFFF ? -1 : best;
    const bool stop = ld >= 0 && d.stop_on_legal;
    if (stop) {
        if (d.cmax > 1) {
            // multicolouring: the legal member's selection as [i][s]
            for (int e = threadIdx.x; e < d.n * d.cmax; e += blockDim.x) {
                const int i = e / d.cmax, sl = e - i * d.cmax;
                d.snap[e] = d.sel[((size_t)ld * d.cmax + sl) * d.cs + i];
            }
        } else {
            const int16_t* c = d.c[p] + (size_t)ld * d.cs;
            for (int i = threadIdx.x; i < d.n; i += blockDim.x) d.snap[i] = c[i];
        }
        if (threadIdx.x == 0) {
            st->legal_d = ld;
            st->stopped = 1;
        }
    }
    if ((flags & kFlagFlipFused) && d.pfuse && threadIdx.x == 0 && !stop) {
        // the sparse-rows launch wrote this iteration's update into the other buffers
        st->pW ^= 1;
        st->pS ^= 1;
    }
    if ((flags & kFlagFused) && threadIdx.x == 0 && !stop) {
        // fused path: the contraction kernel wrote the update into the other buffers
        st->pW ^= 1;
        st->pS ^= 1;
        st->t += 1;
        st->steps_done += 1;
        if (st->next_bad) {
            st->error = -5;
            st->stopped = 1;
        }
    }
}

__global__ __launch_bounds__(256) void k_fitness(const GraphDev* __restrict__ gd, int G, int honor_stop,
                                                 int flags, int gsel) {
    __shared__ int best;
    const int g = blockIdx.x;
    if (g >= G || (gsel >= 0 && g != gsel)) return;
    fitness_graph(gd, g, honor_stop, flags, &best);
}

// Separate-kernel path, step 4: softmax along k, straight-through gradient,
// update and smoothing (mode 0), or gradient output without update (mode 1,
// one graph).  16 lanes per row (d, i).
__global__ __launch_bounds__(256) void k_update(const GraphDev* __restrict__ gd, int G, int total_rows,
                                                int honor_stop, int mode, int gsel,
                                                float* __restrict__ gS_out, float* __restrict__ gW_out) {
    const int l16 = threadIdx.x & 15;
    const int row = blockIdx.x * 16 + (threadIdx.x >> 4);
    if (row >= total_rows) return;
    const int g = graph_of_row(gd, G, row);
    if (gsel >= 0 && g != gsel) return;
    const GraphDev& d = gd[g];
    GraphState* st = d.st;
    if (honor_stop && st->stopped) return;
    const int r = row - d.row_begin;
    const int m = r / d.n;
    const int k = d.k;
    float* w = d.W[0] + (size_t)r * k;
    const float* gs = d.G + (size_t)r * k;
    const long long t = st->t;
    const float nut = prob_added(d.problem) ? d.nu * (float)t : 0.0f;
    const int prob = d.problem;
    const int32_t* V = d.V[st->pS] + (size_t)m * k;
    const float gam = d.momentum;
    float* vel = d.vel ? d.vel + (size_t)r * k : nullptr;
    float mx = -INFINITY;
    for (int l = l16; l < k; l += 16) mx = fmaxf(mx, w[l]);
    mx = row16_max(mx);
    float z = 0.0f, q = 0.0f;
    for (int l = l16; l < k; l += 16) {
        float e = exp_soft(w[l] - mx);
        float gv = gs[l];
        if (nut != 0.0f) gv += nut * added_grad(prob, V[l], l, d.c1, d.c2);
        z += e;
        q += e * gv;
    }
    z = row16_sum(z);
    q = row16_sum(q);
    const float rz = 1.0f / z;
    const float rr = q * rz;
    const bool smooth = d.nb_iter > 0 && ((t + 1) % d.nb_iter) == 0;
    for (int l = l16; l < k; l += 16) {
        float e = exp_soft(w[l] - mx) * rz;
        float gv = gs[l];
        if (nut != 0.0f) gv += nut * added_grad(prob, V[l], l, d.c1, d.c2);
        float gw = e * (gv - rr);
        if (mode == 0) {
            float step = gw;
            if (vel) {
                step = gam * vel[l] + gw;       // heavy-ball velocity
                vel[l] = step;
            }
            float nw = w[l] - d.eta * step;
            if (smooth) nw = nw / d.rho;
            w[l] = nw;
        } else {
            if (gS_out) gS_out[(size_t)r * k + l] = gv;
            if (gW_out) gW_out[(size_t)r * k + l] = gw;
        }
    }
}

// Step 4 with the row held in registers, one (member, vertex) row per 16-lane
// group, k <= 16 KPL: softmax along k (max subtracted), straight-through
// gradient gW = s^ (G - sum_l s^_l G_l), update, smoothing, and in mode 0 the
// argmax colouring of the updated row for the next iteration (written over
// this iteration's colours).  Mode 1 writes gS and gW of graph gsel instead.
// VAR bit 0: some graph of the launch has an added fitness term (equity or colour
// cost), bit 1: some graph takes heavy-ball steps; the plain variant carries neither
// stream's registers.
template <int KPL, int VAR>
__device__ __forceinline__ void update_row(const GraphDev* __restrict__ gd, int G, int row, int honor_stop, int mode,
                                           int gsel, float* __restrict__ gS_out, float* __restrict__ gW_out) {
    const int l16 = threadIdx.x & 15;
    const int g = graph_of_row(gd, G, row);
    if (gsel >= 0 && g != gsel) return;
    const GraphDev& d = gd[g];
    GraphState* st = d.st;
    if (honor_stop && st->stopped) return;
    // the fast path's sparse graphs take their row update in the sparse-rows launch
    if (mode == 0 && d.pfuse) return;
    const int r = row - d.row_begin;
    const int k = d.k;
    const int m = r / d.n, i = r - m * d.n;
    float* w = d.W[0] + (size_t)r * k;
    const float* gs = d.G + (size_t)r * k;
    const long long t = st->t;
    const float nut = prob_added(d.problem) ? d.nu * (float)t : 0.0f;
    const int prob = d.problem;
    const int32_t* V = d.V[st->pS] + (size_t)m * k;
    // fields used after the stores below stay in registers (no reload through gd)
    const int c1 = d.c1, c2 = d.c2;
    const float eta = d.eta, rho = d.rho;
    const float gam = d.momentum;
    float* __restrict__ vel = d.vel ? d.vel + (size_t)r * k : nullptr;
    int16_t* __restrict__ cnext = d.c[st->pS] + (size_t)m * d.cs;
    // every load of the row first (indices clamped into the row inside the last group of
    // 16 instead of per-lane branches, so they are all in flight together), then the
    // arithmetic.  Groups of 16 past the row's end are skipped whole: KPL is sized for the
    // largest k of the launch, and a row of a graph with fewer colours would otherwise
    // issue every group's loads.
    constexpr bool ADD = (VAR & 1) != 0, MOM = (VAR & 2) != 0;
    float wv[KPL], gv[KPL], vv[MOM ? KPL : 1];
    int32_t cv[ADD ? KPL : 1];
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
        if (16 * q < k) {
            const int l = min(l16 + 16 * q, k - 1);
            wv[q] = gview(w)[l];
            gv[q] = gview(gs)[l];
        }
    }
    if constexpr (ADD) {
        if (nut != 0.0f) {
#pragma unroll
            for (int q = 0; q < KPL; ++q)
                if (16 * q < k) cv[q] = gview(V)[min(l16 + 16 * q, k - 1)];
        }
    }
    if constexpr (MOM) {
        if (vel && mode != 1) {
#pragma unroll
            for (int q = 0; q < KPL; ++q)
                if (16 * q < k) vv[q] = gview((const float*)vel)[min(l16 + 16 * q, k - 1)];
        }
    }
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
        const int l = l16 + 16 * q;
        if (l < k) {
            if constexpr (ADD) {
                if (nut != 0.0f) gv[q] += nut * added_grad(prob, cv[q], l, c1, c2);
            }
        } else {
            wv[q] = -INFINITY;
            gv[q] = 0.0f;
        }
    }
    float mx = -INFINITY;
#pragma unroll
    for (int q = 0; q < KPL; ++q) mx = fmaxf(mx, wv[q]);
    mx = row16_max(mx);
    float ev[KPL];
    float z = 0.0f, qs = 0.0f;
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
        ev[q] = (l16 + 16 * q < k) ? exp_soft(wv[q] - mx) : 0.0f;
        z += ev[q];
        qs += ev[q] * gv[q];
    }
    z = row16_sum(z);
    qs = row16_sum(qs);
    const float rz = 1.0f / z;
    const float rq = qs * rz;
    if (mode == 1) {
#pragma unroll
        for (int q = 0; q < KPL; ++q) {
            const int l = l16 + 16 * q;
            if (l < k) {
                if (gS_out) gS_out[(size_t)r * k + l] = gv[q];
                if (gW_out) gW_out[(size_t)r * k + l] = ev[q] * rz * (gv[q] - rq);
            }
        }
        return;
    }
    const bool smooth = d.nb_iter > 0 && ((t + 1) % d.nb_iter) == 0;
    float best = -INFINITY;
    int bi = 0x7FFFFFFF, bad = 0;
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
        const int l = l16 + 16 * q;
        if (l < k) {
            float step = ev[q] * rz * (gv[q] - rq);
            if constexpr (MOM) {
                if (vel) {
                    step = gam * vv[q] + step;  // heavy-ball velocity
                    vel[l] = step;
                }
            }
            float nw = wv[q] - eta * step;
            if (smooth) nw = nw / rho;
            w[l] = nw;
            if (!finite_f(nw)) bad = 1;
            if (nw > best) { best = nw; bi = l; }
        }
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
        cnext[i] = (int16_t)bi;
    }
}

template <int KPL, int VAR>
__global__ __launch_bounds__(256) void k_update_rows(const GraphDev* __restrict__ gd, int G, int total_rows,
                                                     int honor_stop, int mode, int gsel, float* __restrict__ gS_out,
                                                     float* __restrict__ gW_out) {
    const int row = blockIdx.x * 16 + (threadIdx.x >> 4);
    if (row >= total_rows) return;
    update_row<KPL, VAR>(gd, G, row, honor_stop, mode, gsel, gS_out, gW_out);
}

// t <- t + 1 for every graph still running.
__global__ void k_advance(const GraphDev* __restrict__ gd, int G) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    advance_graph(gd[g].st);
}

// FP64 loss of one graph: L = sum main fitness + nu t sum added fitness + lambda t kappa
// - mu t varpi (kappa, varpi from the group-concentration kernel's partials).
__global__ __launch_bounds__(256) void k_loss(const GraphDev* __restrict__ gd, int g, int ntiles,
                                              double* __restrict__ out) {
    __shared__ double red[4][256];
    const GraphDev& d = gd[g];
    double ka = 0, vb = 0, sf = 0, se = 0;
    for (int u = threadIdx.x; u < ntiles; u += 256) {
        ka += d.part[2 * u];
        vb += d.part[2 * u + 1];
    }
    for (int m = threadIdx.x; m < d.D; m += 256) {
        sf += (double)d.fcol[m];
        se += (double)d.feq[m];
    }
    red[0][threadIdx.x] = ka; red[1][threadIdx.x] = vb;
    red[2][threadIdx.x] = sf; red[3][threadIdx.x] = se;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if (threadIdx.x < s)
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double t = (double)d.st->t;
        const double eq = prob_added(d.problem) ? red[3][0] : 0.0;
        out[0] = red[2][0] + (double)d.nu * t * eq + (double)d.lambda * t * red[0][0] - (double)d.mu * t * red[1][0];
        out[1] = red[2][0];
        out[2] = eq;
        out[3] = red[0][0];
        out[4] = red[1][0];
    }
}

// copy fitness / colour outputs of one graph for tcol_conflicts
__global__ void k_copy_report(const GraphDev* __restrict__ gd, int g, int16_t* colors, int64_t* fcol,
                              int64_t* feq) {
    const GraphDev& d = gd[g];
    const int p = d.st->pS;
    const size_t total = (size_t)d.D * d.n;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        if (colors) {
            const size_t m = e / d.n;
            colors[e] = d.c[p][m * d.cs + (e - m * d.n)];
        }
        if (e < (size_t)d.D) {
            if (fcol) fcol[e] = d.fcol[e];
            if (feq) feq[e] = d.feq[e];
        }
    }
}

// graph g's selection as [d][i][s]: the cmax colours of each vertex (slot 0 the argmax, -1 past
// the demand), or the argmax colouring when cmax = 1
__global__ void k_copy_selection(const GraphDev* __restrict__ gd, int g, int16_t* __restrict__ out) {
    const GraphDev& d = gd[g];
    const int CM = d.cmax, n = d.n;
    const int16_t* c = d.c[d.st->pS];
    const size_t total = (size_t)d.D * n * CM;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const size_t mi = e / CM;
        const int sl = (int)(e - mi * CM);
        const size_t m = mi / n, i = mi - m * n;
        out[e] = CM > 1 ? d.sel[((size_t)m * CM + sl) * d.cs + i] : c[m * d.cs + i];
    }
}

__global__ void k_state(const GraphDev* __restrict__ gd, int G, int op, int g_only, long long t) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G || (g_only >= 0 && g != g_only)) return;
    GraphState* st = gd[g].st;
    if (op == 0) {            // reset run state (keeps t and the route counters)
        st->stopped = 0; st->error = 0; st->legal_d = -1; st->steps_done = 0; st->next_bad = 0;
        st->prep_ticket = 0;
    } else if (op == 1) {     // set t
        st->t = t;
    } else if (op == 2) {     // clear steps counter only
        st->steps_done = 0; st->legal_d = -1;
    } else if (op == 3) {     // the caller's buffer holds the weights again
        st->pW = 0;
    } else if (op == 4) {     // clear the conflict accumulators (after timing repeated contractions)
        for (int m = 0; m < gd[g].D; ++m) gd[g].f2[m] = 0;
    } else if (op == 5) {     // the sparse rows' route for this iteration (timing of its contraction form)
        st->pdense = 0;
    }
}

// ------------------------------------------------------------ initial weights -

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11), from its published round
// function and constants: ten rounds of two 32x32->64 multiplies, with the key
// bumped by the Weyl constants between rounds.
__device__ inline void philox4x32_10(uint32_t (&x)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)x[0] * 0xD2511F53ull;
        const uint64_t p1 = (uint64_t)x[2] * 0xCD9E8D57ull;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ x[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ x[3] ^ k1;
        x[0] = n0;
        x[1] = (uint32_t)p1;
        x[2] = n2;
        x[3] = (uint32_t)p0;
    }
}

// two 32-bit words to a uniform in (0, 1] with 53 bits
__device__ inline double uniform53(uint32_t hi, uint32_t lo) {
    return ((double)(hi >> 5) * 67108864.0 + (double)(lo >> 6) + 1.0) * (1.0 / 9007199254740992.0);
}

// W[e] ~ N(0, sigma0^2), e < count: counter block b = (b mod 2^32, b / 2^32, stream 1, 0)
// under key = seed gives two uniforms (u1, u2) and, by Box-Muller in FP64, the normals
// r cos(2 pi u2) and r sin(2 pi u2), r = sqrt(-2 ln u1), for entries 2b and 2b+1,
// scaled by sigma0 and rounded to fp32.  One thread per block b.
__global__ __launch_bounds__(256) void k_init_weights(float* __restrict__ W, long long count, uint32_t key0,
                                                      uint32_t key1, double sigma0) {
    const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (2 * b >= count) return;
    uint32_t x[4] = {(uint32_t)b, (uint32_t)((unsigned long long)b >> 32), 1u, 0u};
    philox4x32_10(x, key0, key1);
    const double u1 = uniform53(x[0], x[1]), u2 = uniform53(x[2], x[3]);
    const double r = sqrt(-2.0 * log(u1));
    const double th = 6.283185307179586 * u2;
    W[2 * b] = (float)(r * cos(th) * sigma0);
    if (2 * b + 1 < count) W[2 * b + 1] = (float)(r * sin(th) * sigma0);
}

// ------------------------------------------------ class-conflict matrix ---------

// C_d = S_d^T (A.S_d) for one graph on fp32 MFMA (16x16x4; the integer entries stay below
// 2^24, so the FP32 accumulation is exact): the A operand is the one-hot S_d^T, made in
// registers from the colours (row l, column i: 1 when c_d(i) = l), the B operand the
// contraction's A.S_d from G ([D][n][k], rows i, columns l').  A block of 4 waves takes
// member d = blockIdx.z, rows l0 .. l0 + 15 (blockIdx.y) and columns 64 blockIdx.x .. + 63,
// one 16 x 16 tile per wave; out is [D][k][k] int32.
typedef float f32x4k __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_class_conflicts(const GraphDev* __restrict__ gd, int g,
                                                         int32_t* __restrict__ out) {
    const GraphDev& d = gd[g];
    const int k = d.k, n = d.n;
    const int dm = blockIdx.z;
    const int l0 = blockIdx.y * 16;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c0 = blockIdx.x * 64 + wave * 16;
    if (c0 >= k) return;
    const int16_t* __restrict__ col = d.c[d.st->pS] + (size_t)dm * d.cs;
    const float* __restrict__ Gd = d.G + (size_t)dm * n * k;
    const int lrow = l0 + (lane & 15);          // A operand row (colour l)
    const int ccol = c0 + (lane & 15);          // B operand column (colour l')
    const int kk = lane >> 4;                   // K index within the step
    f32x4k acc = {0.f, 0.f, 0.f, 0.f};
    constexpr int U = 8;                        // K-steps of 4 per round of loads
    for (int i0 = 0; i0 < n; i0 += 4 * U) {
        float a[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + 4 * u + kk;
            const bool in = i < n;
            const int ci = in ? (int)gview(col)[i] : -1;
            a[u] = ci == lrow ? 1.0f : 0.0f;
            b[u] = (in && ccol < k) ? gview(Gd)[(size_t)i * k + ccol] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], b[u], acc, 0, 0, 0);
    }
    // lane holds rows 4 (lane / 16) + r, column lane mod 16 of the tile; G holds -A.S for
    // partitioning
    const float sg = prob_partition(d.problem) ? -1.0f : 1.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int l = l0 + (lane >> 4) * 4 + r, lp = c0 + (lane & 15);
        if (l < k && lp < k) out[((size_t)dm * k + l) * k + lp] = (int32_t)(sg * acc[r]);
    }
}

// ------------------------------------------- descriptors from kernel arguments --

// Writes one graph's descriptor and a fresh state (the values travel as kernel arguments,
// so a captured launch carries them; no host buffer has to outlive the call).
__global__ void k_put_desc(GraphDev d, GraphDev* __restrict__ gd, GraphState* __restrict__ st) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    *gd = d;
    GraphState s{};
    s.legal_d = -1;
    *st = s;
}

// p[0 .. words) = 0 (16-byte stores; p 16-byte aligned)
__global__ __launch_bounds__(256) void k_zero16(uint4* __restrict__ p, size_t words) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < words; e += (size_t)gridDim.x * blockDim.x)
        p[e] = make_uint4(0u, 0u, 0u, 0u);
}

// ------------------------------------------------------------- launchers -----

#define TCOL_LAUNCH_CHECK() do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

hipError_t launch_init_weights(float* W, long long count, unsigned long long seed, double sigma0, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const long long blocks = ((count + 1) / 2 + 255) / 256;
    hipLaunchKernelGGL(k_init_weights, dim3((unsigned)blocks), dim3(256), 0, s, W, count, (uint32_t)seed,
                       (uint32_t)(seed >> 32), sigma0);
    TCOL_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_pack_graph(const uint8_t* A, int n, int n_pad, int prec, uint8_t* A8, void* Aop, int* bad,
                             unsigned long long* ones, hipStream_t s) {
    const long long total = (long long)n_pad * n_pad;
    const int blocks = (int)std::min<long long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_pack_graph, dim3(blocks), dim3(256), 0, s, A, n, n_pad, prec, A8, Aop, bad, ones);
    TCOL_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_colors(const GraphDev* gd, int G, int total_rows, int honor_stop, hipStream_t s) {
    if (total_rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_colors, dim3(ceil_div(total_rows, 16)), dim3(256), 0, s, gd, G, total_rows, honor_stop);
    TCOL_LAUNCH_CHECK();
    return hipSuccess;
}

size_t prep_lds(int kmax, int nmax, int lists) {
    size_t b = sizeof(int) * ((size_t)kPrepScratch + (size_t)kmax);
    if (lists) b += sizeof(int) * 5 * (size_t)kmax + sizeof(int16_t) * (size_t)nmax;
    return (b + 15) / 16 * 16;
}

hipError_t launch_prep(const GraphDev* gd, int G, int total_mem, size_t lds, int honor_stop, int next, int decide,
                       int ex_blocks, int advance_prev, hipStream_t s) {
    if (total_mem <= 0) return hipSuccess;
    if (lds > 150 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_prep, dim3(total_mem + ex_blocks), dim3(256), lds, s, gd, G, total_mem, honor_stop, next,
                       decide, ex_blocks, advance_prev);
    TCOL_LAUNCH_CHECK();
    return hipSuccess;
}

// instantiations of the sparse rows: KW = 0 (no row update), or the row update's values per lane
// (k <= 64 KW) for graphs whose update rides on the launch, with (ADD = 1) or without the added
// fitness term (the equity or colour-cost gradient, whose class-size loads take registers)
#define TCOL_PS_KERNELS(X) \
    X(256, 0, 0) X(512, 0, 0) X(1024, 0, 0) \
    X(512, 2, 0) X(512, 3, 0) X(512, 5, 0) X(512, 7, 0) X(512, 9, 0) \
    X(512, 2, 1) X(512, 3, 1) X(512, 5, 1) X(512, 7, 1) X(512, 9, 1) \
    X(1024, 2, 0) X(1024, 3, 0) X(1024, 5, 0) X(1024, 7, 0) X(1024, 9, 0) \
    X(1024, 2, 1) X(1024, 3, 1) X(1024, 5, 1) X(1024, 7, 1) X(1024, 9, 1)

int penalty_sparse_kw(int kmax) {
    for (int kw : {2, 3, 5, 7, 9})
        if (64 * kw >= kmax) return kw;
    return -1;
}

hipError_t penalty_sparse_prepare() {
#define TCOL_PS_ATTR(NT, KW, ADD)                                                                            \
    {                                                                                                        \
        const hipError_t e = hipFuncSetAttribute((const void*)k_pen_sparse<NT, KW, ADD>,                     \
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);    \
        if (e != hipSuccess) return e;                                                                       \
    }
    TCOL_PS_KERNELS(TCOL_PS_ATTR)
#undef TCOL_PS_ATTR
    // k_prep also holds 1 KB of static LDS
    return hipFuncSetAttribute((const void*)k_prep, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
}

size_t penalty_sparse_lds(int PM, int kmax, int dmax, int nmax) {
    const size_t n_pad = (size_t)round_up(nmax, kPadN);
    const size_t acc = 8 * (size_t)PM * (size_t)kmax;
    const size_t work = acc > 4 * n_pad ? acc : 4 * n_pad;
    const size_t b = 8 * ps_tab_words(dmax) + 2 * 4 * ps_int_words(dmax) + 16 + 2 * (size_t)round_up(dmax, 8) +
                     4 * n_pad + work;
    return (b + 15) / 16 * 16;
}

hipError_t launch_penalty_sparse(const GraphDev* gd, int G, int blocks, int PM, int threads, int kw, int add,
                                 size_t lds, int honor_stop, int accumulate, hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    const int grid = blocks;
    if (PM != 8 || lds > 160 * 1024) return hipErrorInvalidValue;
    // the fused row update takes one wave per member of a group
    if (kw > 0 && PM > threads / 64) return hipErrorInvalidValue;
    bool done = false;
    if (kw == 0) add = 0;
#define TCOL_PS_LAUNCH(NT, KW, ADD)                                                                         \
    if (!done && threads == NT && kw == KW && add == ADD) {                                                 \
        k_pen_sparse<NT, KW, ADD><<<grid, NT, lds, s>>>(gd, G, blocks, honor_stop, PM, accumulate);         \
        done = true;                                                                                        \
    }
    TCOL_PS_KERNELS(TCOL_PS_LAUNCH)
#undef TCOL_PS_LAUNCH
    if (!done) return hipErrorInvalidValue;
    TCOL_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_expand(const GraphDev* gd, int G, int total_blocks, int honor_stop, int next, int gate,
                         hipStream_t s) {
    if (total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_expand, dim3(total_blocks), dim3(256), 0, s, gd, G, total_blocks, honor_stop, next, gate);
    TCOL_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_mtilde(const GraphDev* gd, int G, int total_tiles, int honor_stop, int flags, int gsel,
                         int32_t* mt_out, hipStream_t s) {
    if (total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mtilde, dim3(total_tiles), dim3(256), 0, s, gd, G, total_tiles, honor_stop, flags, gsel,
                       mt_out);
    TCOL_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_fitness(const GraphDev* gd, int G, int honor_stop, int flags, int gsel, hipStream_t s) {
    hipLaunchKernelGGL(k_fitness, dim3(G), dim3(256), 0, s, gd, G, honor_stop, flags, gsel);
    TCOL_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_update(const GraphDev* gd, int G, int total_rows, int honor_stop, int mode, int gsel,
                         float* gS_out, float* gW_out, hipStream_t s) {
    if (total_rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_update, dim3(ceil_div(total_rows, 16)), dim3(256), 0, s, gd, G, total_rows, honor_stop,
                       mode, gsel, gS_out, gW_out);
    TCOL_LAUNCH_CHECK();
    return hipSuccess;
}

int update_rows_kpl(int kmax) {
    const int need = (kmax + 15) / 16;
    for (int kpl : {2, 4, 6, 8, 12, 18, 24, 36})
        if (kpl >= need) return kpl;
    return 0;
}

hipError_t launch_update_rows(const GraphDev* gd, int G, int total_rows, int kmax, int var, int honor_stop, int mode,
                              int gsel, float* gS_out, float* gW_out, hipStream_t s) {
    if (total_rows <= 0) return hipSuccess;
    if (var < 0 || var > 3) return hipErrorInvalidValue;
    const dim3 grid(ceil_div(total_rows, 16)), blk(256);
#define TCOL_UR(KP)                                                                                                  \
    switch (var) {                                                                                                   \
        case 0: hipLaunchKernelGGL((k_update_rows<KP, 0>), grid, blk, 0, s, gd, G, total_rows, honor_stop, mode, gsel, \
                                   gS_out, gW_out); break;                                                           \
        case 1: hipLaunchKernelGGL((k_update_rows<KP, 1>), grid, blk, 0, s, gd, G, total_rows, honor_stop, mode, gsel, \
                                   gS_out, gW_out); break;                                                           \
        case 2: hipLaunchKernelGGL((k_update_rows<KP, 2>), grid, blk, 0, s, gd, G, total_rows, honor_stop, mode, gsel, \
                                   gS_out, gW_out); break;                                                           \
        default: hipLaunchKernelGGL((k_update_rows<KP, 3>), grid, blk, 0, s, gd, G, total_rows, honor_stop, mode, gsel, \
                                    gS_out, gW_out); break;                                                          \
    }
    switch (update_rows_kpl(kmax)) {
        case 2: TCOL_UR(2) break;
        case 4: TCOL_UR(4) break;
        case 6: TCOL_UR(6) break;
        case 8: TCOL_UR(8) break;
        case 12: TCOL_UR(12) break;
        case 18: TCOL_UR(18) break;
        case 24: TCOL_UR(24) break;
        case 36: TCOL_UR(36) break;
        default: return hipErrorInvalidValue;
    }
#undef TCOL_UR
    TCOL_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_advance(const GraphDev* gd, int G, hipStream_t s) {
    hipLaunchKernelGGL(k_advance, dim3(ceil_div(G, 64)), dim3(64), 0, s, gd, G);
    TCOL_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_loss(const GraphDev* gd, int g, int ntiles, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, s, gd, g, ntiles, out);
    TCOL_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_copy_report(const GraphDev* gd, int g, int16_t* colors, int64_t* fcol, int64_t* feq,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_copy_report, dim3(256), dim3(256), 0, s, gd, g, colors, fcol, feq);
    TCOL_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_class_conflicts(const GraphDev* gd, int g, int D, int k, int32_t* out, hipStream_t s) {
    if (D <= 0 || k <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_class_conflicts, dim3(ceil_div(k, 64), ceil_div(k, 16), D), dim3(256), 0, s, gd, g, out);
    TCOL_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_put_desc(const GraphDev& d, GraphDev* gd, GraphState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, s, d, gd, st);
    TCOL_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    if (((uintptr_t)p & 15) || (bytes & 15)) return hipErrorInvalidValue;
    const size_t words = bytes / 16;
    const int blocks = (int)std::min<size_t>((words + 255) / 256, 2048);
    hipLaunchKernelGGL(k_zero16, dim3(blocks), dim3(256), 0, s, (uint4*)p, words);
    TCOL_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_copy_selection(const GraphDev* gd, int g, int16_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_selection, dim3(512), dim3(256), 0, s, gd, g, out);
    TCOL_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_state(const GraphDev* gd, int G, int op, int g_only, long long t, hipStream_t s) {
    hipLaunchKernelGGL(k_state, dim3(ceil_div(G, 64)), dim3(64), 0, s, gd, G, op, g_only, t);
    TCOL_LAUNCH_CHECK();
    return hipSuccess;
}

}  // namespace tcol
