// Batched AB-/BA-GMRES (Sec. 2) over many independent problems of different geometry.
//
// One round advances every running problem by one Arnoldi step with a fixed sequence of
// persistent kernels, captured once in a HIP graph and replayed every round:
//
//   begin     per problem: the step to run (0: sits out), and the work lists of the round
//   pad       BA: w_k -> padded image copies       AB: t = B w_k -> padded copies
//   forward   BA: z = A w_k                        AB: q = A t
//   back      AB: t = B w_k                        BA: q = B z
//   mgs       modified Gram-Schmidt, one block group per problem (group barriers)
//   givens    FP64 Givens update and y_k, one block per problem
//   residual  ||r_k|| (BA: (b - A x0) - Z y_k; AB: W_{k+1}(beta e_1 - H y)) and the DP
//             candidate test
//
// The work lists live in device memory and are rebuilt by `begin` every round, so the
// graph never changes while problems join and leave (two variants are kept: the AB and
// BA projector chains in sequence, or as two branches while the problems are small). Blocks take work items from a
// per-list ticket counter; an item's arithmetic depends only on its own problem, so a
// problem's results are the same alone and in any mix.
//
// The host reads a copy of the per-problem scalars one round behind. A DP candidate, a
// breakdown or the iteration cap holds the problem (its later rounds skip it); the host
// then enqueues the formation of x_k and the explicit residual ||b - A x_k||, and a small
// kernel accepts the candidate or resumes the problem. Nothing waits on the host except
// the one-round-behind copy.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <vector>

#include "krylov_body.h"
#include "back_body.h"
#include "fwd_body.h"

namespace abg {

// Work lists are split into kRanges contiguous ranges with a counter each (see
// for_each_item); the list-order schedule claims at most kMaxListChunk items at a time.
constexpr int kRanges = 8;
constexpr int kMaxListChunk = 8;

enum Tab {
    kTPadBA = 0,   // pad w_k (BA)
    kTBackAB,      // t = B w_k (AB), interpolating back projector
    kTBackABAdj,   // t = A^T w_k (AB), matched pair
    kTFwdBA,       // z = A w_k (BA)
    kTPadAB,       // pad t (AB)
    kTBackBA,      // q = B z (BA), interpolating back projector
    kTBackBAAdj,   // q = A^T z (BA), matched pair
    kTFwdAB,       // q = A t (AB)
    kTMgsS,        // MGS groups with the small register tile
    kTMgsL,        // MGS groups with the large register tile
    kTMgsH,        // MGS groups with the largest register tile (FP32/BF16 basis)
    kTMgsX,        // streaming MGS groups (vectors the register tiles cannot hold)
    kTRes,         // residual chunks
    kTGiv,         // one Givens block per problem
    kNumTab
};

constexpr int kMgsSmallE = 8;
constexpr int kMgsLargeE = 32;
constexpr int kMgsHugeE = 64;
constexpr int kMgsSmallMaxG = 128;
constexpr int kMgsStreamG = 512;
constexpr int kResU = 4;

// Per-problem descriptor in device memory.
struct BatchInst {
    const AngleParams *ang;
    int N, S, n_ang, n_det;
    double ds, s0;
    int method, kind, k_max, ld;
    long long L, ldv, mp, n, m;
    void *V, *Z, *cur, *q, *rb0, *tm, *tn, *xr, *xc;
    double *H, *R, *cs, *sn, *g, *Y, *rho, *part, *mgs_part, *q64;
    unsigned *count;
    double bd_rel;
    int mgs_rows;
    int need_res;
    int mgs_G, mgs_class;   // register tile class 0 small, 1 large, 3 huge; 2 streaming
    int chunk, n_chunks;
    int fwd_rays;           // forward block shape of the single-solve rule (tiles.rays = 0)
};

// Work lists: list t holds segments (problem, first ticket); items of a segment are
// consecutive tickets.
struct TabView {
    int *nseg, *total;
    unsigned *ticket;    // [kNumTab][kRanges]
    int *slot, *first;   // [kNumTab][max_slots]
    int max_slots;
    __device__ int seg_slot(int t, int i) const { return slot[t * max_slots + i]; }
    __device__ int seg_first(int t, int i) const { return first[t * max_slots + i]; }
};

struct Tiles {
    int rays;        // forward projector: rays of one angle per block (64, 128 or 256);
                     // a block of 256 threads takes 256/rays angles; 0: per problem, the
                     // shape single solves of its geometry use
    int ang_block;   // back projectors: angles staged in LDS per round (64 or 128)
    int sched;       // item schedule of the projector and residual lists (for_each_item)
    int stage = 0;   // eighths of the four-angle forward items that stage their band rows
                     // in LDS (set at launch from the single-solve rule)
};

namespace {

__device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

__device__ int items_of(int t, const BatchInst &d, const Tiles &tl)
{
    const bool ba = d.method == ABG_METHOD_BA;
    switch (t) {
    case kTPadBA: return ba ? ceil_div(d.N, 32) * ceil_div(d.N, 32) : 0;
    case kTPadAB: return ba ? 0 : ceil_div(d.N, 32) * ceil_div(d.N, 32);
    case kTBackAB:
    case kTBackABAdj:
    case kTBackBA:
    case kTBackBAAdj: {
        const bool want_ba = t == kTBackBA || t == kTBackBAAdj;
        const bool want_adj = t == kTBackABAdj || t == kTBackBAAdj;
        if (ba != want_ba || (d.kind == ABG_BP_ADJ) != want_adj) return 0;
        return ceil_div(d.N, kTile) * ceil_div(d.N, kTile);
    }
    case kTFwdBA:
    case kTFwdAB: {
        if ((t == kTFwdBA) != ba) return 0;
        const int rays = tl.rays ? tl.rays : d.fwd_rays;
        return ceil_div(d.n_ang, 256 / rays) * ceil_div(d.n_det, rays);
    }
    case kTMgsS: return d.mgs_class == 0 ? d.mgs_G : 0;
    case kTMgsL: return d.mgs_class == 1 ? d.mgs_G : 0;
    case kTMgsX: return d.mgs_class == 2 ? d.mgs_G : 0;
    case kTMgsH: return d.mgs_class == 3 ? d.mgs_G : 0;
    case kTRes: return d.need_res ? d.n_chunks : 0;
    case kTGiv: return 1;
    }
    return 0;
}

// ---- begin ------------------------------------------------------------------------------
// Block t builds list t; block 0 also publishes each problem's step for the round.
__global__ __launch_bounds__(256) void begin_kernel(const BatchInst *__restrict__ D, DevState *S, TabView tv,
                                                    int n_slots, Tiles tl)
{
    __shared__ int wsum_n[4], wsum_c[4];
    const int t = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int per = (n_slots + 255) / 256;
    const int s_lo = min(tid * per, n_slots), s_hi = min(s_lo + per, n_slots);
    int my_n = 0, my_c = 0;
    for (int s = s_lo; s < s_hi; ++s) {
        const DevState &st = S[s];
        const BatchInst &d = D[s];
        const bool run = st.active && !st.done && !st.stop && !st.error &&
                         !(st.bd_k != 0 && st.bd_k <= st.k) && st.k < d.k_max;
        const int kc = run ? st.k + 1 : 0;
        if (t == 0) S[s].kcur = kc;
        const int c = kc ? items_of(t, d, tl) : 0;
        my_n += c > 0;
        my_c += c;
    }
    // exclusive block scan of (segments, items)
    int in = my_n, ic = my_c;
    for (int o = 1; o < 64; o <<= 1) {
        const int a = __shfl_up(in, o, 64), b = __shfl_up(ic, o, 64);
        if (lane >= o) {
            in += a;
            ic += b;
        }
    }
    if (lane == 63) {
        wsum_n[w] = in;
        wsum_c[w] = ic;
    }
    __syncthreads();
    int base_n = 0, base_c = 0, tot_n = 0, tot_c = 0;
    for (int i = 0; i < 4; ++i) {
        if (i < w) {
            base_n += wsum_n[i];
            base_c += wsum_c[i];
        }
        tot_n += wsum_n[i];
        tot_c += wsum_c[i];
    }
    int on = base_n + in - my_n, oc = base_c + ic - my_c;
    for (int s = s_lo; s < s_hi; ++s) {
        const DevState &st = S[s];
        const BatchInst &d = D[s];
        const bool run = st.active && !st.done && !st.stop && !st.error &&
                         !(st.bd_k != 0 && st.bd_k <= st.k) && st.k < d.k_max;
        const int c = run ? items_of(t, d, tl) : 0;
        if (c > 0) {
            tv.slot[t * tv.max_slots + on] = s;
            tv.first[t * tv.max_slots + on] = oc;
            ++on;
            oc += c;
        }
    }
    if (tid == 0) {
        tv.nseg[t] = tot_n;
        tv.total[t] = tot_c;
    }
    if (tid < kRanges) tv.ticket[t * kRanges + tid] = 0u;
}

// Problem and item of ticket `it` of list t (binary search over the segments). Every
// thread of a block calls it with the same ticket, so the loads are uniform.
__device__ inline void locate(const TabView &tv, int t, int it, int *slot, int *local)
{
    int lo = 0, hi = tv.nseg[t] - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tv.seg_first(t, mid) <= it) lo = mid;
        else hi = mid - 1;
    }
    *slot = __builtin_amdgcn_readfirstlane(tv.seg_slot(t, lo));
    *local = __builtin_amdgcn_readfirstlane(it - tv.seg_first(t, lo));
}

// Runs body(slot, local) for the items of list t that this block takes, under one of three
// schedules (a tunable):
//  sched 0  static round-robin: block b takes items b, b + grid, b + 2 grid, ...
//  sched 1  the list is cut into kRanges contiguous ranges with a counter each; block b
//           starts on range b % kRanges (blocks are dispatched round-robin over the XCDs,
//           so each XCD works mostly on its own contiguous part of the list and keeps it
//           in its L2), takes chunks of items from it as it frees up, then helps with the
//           other ranges: items of unequal cost are balanced dynamically. Chunks are
//           guided: a claim takes half of what is left of the range divided by the blocks
//           that start on it, so the last items go one at a time and a phase does not
//           wait on one block's large final chunk (an item of a 2048^2 problem is ~0.1 ms).
//  sched 2  list order: block b takes item b, then the blocks claim the items after the
//           first `grid` through one counter in guided chunks (what is left over twice
//           the grid, between 1 and kMaxListChunk items). The running blocks all work on
//           the same one or two problems, as the blocks of a single solve's launch do, so
//           only those problems' images and sinograms compete for the caches (with one
//           range per XCD, or with chunks of ~100 items, eight or more large problems are
//           in flight at once, more than the Infinity Cache holds, and a served batch ran
//           15% slower); a list no longer than the grid takes no claim at all.
// The pad and residual lists (uniform, cheap items) always run sched 0.
// A block's items come in increasing order, so the segment (problem) of an item is found
// by moving a cursor forward. body must be called by the whole block (it may
// synchronise).
template <typename F>
__device__ inline void for_each_item(const TabView &tv, int t, int sched, F &&body)
{
    __shared__ int s_c, s_len;
    const int total = tv.total[t];
    if ((int)blockIdx.x >= total) return;
    const int nseg = tv.nseg[t];
    int seg = 0;
    auto visit = [&](int it) {
        while (seg + 1 < nseg && tv.seg_first(t, seg + 1) <= it) ++seg;
        body(__builtin_amdgcn_readfirstlane(tv.seg_slot(t, seg)),
             __builtin_amdgcn_readfirstlane(it - tv.seg_first(t, seg)));
    };
    if (sched == 0) {
        for (int it = blockIdx.x; it < total; it += gridDim.x) visit(it);
        return;
    }
    const int G = min((int)gridDim.x, total);
    if (sched == 2) {
        visit(blockIdx.x);
        const int rest = total - G;
        if (rest <= 0) return;
        unsigned *tk = tv.ticket + t * kRanges;
        for (;;) {
            __syncthreads();
            if (threadIdx.x == 0) {
                int c = rest, len = 0;
                const int seen =
                    (int)__hip_atomic_load(tk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (seen < rest) {
                    len = min(kMaxListChunk, max(1, (rest - seen) / (2 * G)));
                    c = (int)__hip_atomic_fetch_add(tk, (unsigned)len, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
                }
                s_c = c;
                s_len = len;
            }
            __syncthreads();
            const int c = __builtin_amdgcn_readfirstlane(s_c);
            if (c >= rest) return;
            const int e = min(rest, c + __builtin_amdgcn_readfirstlane(s_len));
            for (int it = G + c; it < G + e; ++it) visit(it);
        }
    }
    const int per_range = max(1, G / kRanges);
    const int home = (int)(blockIdx.x % kRanges);
    unsigned *tk = tv.ticket + t * kRanges;
    for (int p = 0; p < kRanges; ++p) {
        const int r = (home + p) % kRanges;
        const int lo = (int)((long long)total * r / kRanges);
        const int n = (int)((long long)total * (r + 1) / kRanges) - lo;
        if (r < home) seg = 0;   // wrapped round to an earlier range
        for (;;) {
            __syncthreads();
            if (threadIdx.x == 0) {
                int c = n, len = 0;
                const int seen =
                    (int)__hip_atomic_load(tk + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (seen < n) {
                    len = max(1, (n - seen) / (2 * per_range));
                    c = (int)__hip_atomic_fetch_add(tk + r, (unsigned)len, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
                }
                s_c = c;
                s_len = len;
            }
            __syncthreads();
            const int c = __builtin_amdgcn_readfirstlane(s_c);
            if (c >= n) break;
            const int e = min(n, c + __builtin_amdgcn_readfirstlane(s_len));
            for (int it = lo + c; it < lo + e; ++it) visit(it);
        }
    }
}

// Takes the next ticket of list t for the block: returns false when the list is used up.
// Used where items must be taken in order by running blocks (the MGS block groups).
__device__ inline bool next_item(const TabView &tv, int t, int *slot_out, int *local_out)
{
    __shared__ int s_slot, s_local;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned it = __hip_atomic_fetch_add(tv.ticket + t * kRanges, 1u,
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int slot = -1, local = 0;
        if ((int)it < tv.total[t]) {
            int lo = 0, hi = tv.nseg[t] - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (tv.seg_first(t, mid) <= (int)it) lo = mid;
                else hi = mid - 1;
            }
            slot = tv.seg_slot(t, lo);
            local = (int)it - tv.seg_first(t, lo);
        }
        s_slot = slot;
        s_local = local;
    }
    __syncthreads();
    // the same in every lane: keep it (and what is loaded through it) in scalar registers
    *slot_out = __builtin_amdgcn_readfirstlane(s_slot);
    *local_out = __builtin_amdgcn_readfirstlane(s_local);
    return *slot_out >= 0;
}

template <typename T> __device__ inline T *zcol(const BatchInst &d, int k)
{
    return d.Z ? gfield<T>(d.Z) + (size_t)(k - 1) * d.mp : gfield<T>(d.tm);
}

// ---- projector phases ---------------------------------------------------------------------
// mode 0: BA, w_k;  mode 1: AB, t
template <typename T>
__global__ __launch_bounds__(256) void bpad_kernel(const BatchInst *__restrict__ D, const DevState *S,
                                                   TabView tv, int t, int mode, Tiles tl)
{
    __shared__ PadLds<T> lds;
    // uniform, cheap items: static round-robin
    for_each_item(tv, t, 0, [&](int slot, int local) {
        const BatchInst &d = D[slot];
        const DevState *st = S + slot;
        if (halted(st, st->kcur)) return;
        const int tpr = (d.N + 31) / 32;
        const T *src = mode == 0 ? gfield<const T>(d.cur) : gfield<const T>(d.tn);
        __syncthreads();   // the previous tile's LDS reads are done
        pad_transpose_tile(src, gfield<T>(d.xr), gfield<T>(d.xc), d.N, d.S,
                           (local % tpr) * 32, (local / tpr) * 32, lds);
    });
}

// mode 0: BA, z = A w_k (column k of Z);  mode 1: AB, q = A t
template <typename T>
__global__ __launch_bounds__(256, 8) void bfwd_kernel(const BatchInst *__restrict__ D, const DevState *S,
                                                   TabView tv, int t, int mode, Tiles tl)
{
    __shared__ FwdStageLds<T> lds;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    for_each_item(tv, t, tl.sched, [&](int slot, int local) {
        const BatchInst &d = D[slot];
        const DevState *st = S + slot;
        const int k = st->kcur;
        if (halted(st, k)) return;
        const int rays = tl.rays ? tl.rays : d.fwd_rays;
        const int wpa = rays / 64;       // waves per angle
        const int apb = 256 / rays;      // angles per block
        const int nrg = (d.n_det + rays - 1) / rays;
        // a share of the four-angle items, spread by a hash of the item, walks with its band
        // rows staged in LDS (the whole block, before any wave leaves)
        if (rays == 64 && tl.stage > 0 &&
            (int)(((unsigned)local * 0x9E3779B1u + (unsigned)slot * 0x85EBCA6Bu) >> 29) < tl.stage) {
            T *y = mode == 0 ? zcol<T>(d, k) : gfield<T>(d.q);
            forward_block_staged(gfield<const T>(d.xr), gfield<const T>(d.xc), y,
                                 gfield<const AngleParams>(d.ang), (local / nrg) * 4,
                                 (local % nrg) * 64, d.N, d.S, d.n_ang, d.n_det, d.ds, d.s0, lds);
            return;
        }
        const int a = (local / nrg) * apb + wave / wpa;
        const int i = (local % nrg) * rays + (wave % wpa) * 64 + lane;
        if (a >= d.n_ang) return;   // whole waves
        T *y = mode == 0 ? zcol<T>(d, k) : gfield<T>(d.q);
        forward_ray(gfield<const T>(d.xr), gfield<const T>(d.xc), y,
                    gfield<const AngleParams>(d.ang), a, i, d.N, d.S, d.n_det, d.ds, d.s0);
    });
}

// mode 0: AB, t = B w_k;  mode 1: BA, q = B z. One kernel per back projector kind (their
// lists are separate): with both kinds in one kernel it took 102-144 VGPRs and ran at
// half the occupancy of the single-solve kernel. Launch bounds (waves per SIMD) at the
// single-solve kernel's occupancy where the item loop still fits without spilling, for
// 64 staged angles: the interpolating kind 8 (FP32, 64 VGPRs) and 6 (FP64, 80 VGPRs),
// the matched pair 6 and 4. With 128 staged angles the LDS stage limits the occupancy.
template <typename T, int AB, bool ADJ>
constexpr int kBBackMinWaves = AB != 64 ? 1 : sizeof(T) == 4 ? (ADJ ? 6 : 8) : (ADJ ? 4 : 6);
template <typename T, int AB, bool ADJ>
__global__ __launch_bounds__(kBackThreads, (kBBackMinWaves<T, AB, ADJ>)) void bback_kernel(
    const BatchInst *__restrict__ D, const DevState *S, TabView tv, int t, int mode, Tiles tl)
{
    __shared__ BackLds<T, AB> lds;
    for_each_item(tv, t, tl.sched, [&](int slot, int local) {
        const BatchInst &d = D[slot];
        const DevState *st = S + slot;
        const int k = st->kcur;
        if (halted(st, k)) return;
        const int tpr = (d.N + kTile - 1) / kTile;
        const int c0 = (local % tpr) * kTile, r0 = (local / tpr) * kTile;
        const T *y = mode == 0 ? gfield<const T>(d.cur) : zcol<T>(d, k);
        T *x = mode == 0 ? gfield<T>(d.tn) : gfield<T>(d.q);
        const AngleParams *ang = gfield<const AngleParams>(d.ang);
        back_tile<T, ADJ, AB>(y, x, ang, d.N, d.n_ang, d.n_det, d.ds, d.s0, c0, r0, lds);
    });
}

// ---- Gram-Schmidt, Givens, residual -------------------------------------------------------
// A ticket is one rank of a problem's block group; a group's tickets are consecutive, so
// every group whose first rank is taken is completed by blocks that are running (each
// group is smaller than the grid).
template <typename TX, typename TV, int E>
__global__ __launch_bounds__(kBlock) void bmgs_kernel(const BatchInst *__restrict__ D, DevState *S,
                                                      TabView tv, int t)
{
    __shared__ double lds[kWaves];
    // at most `total` blocks can hold a ticket: the others leave without touching the
    // counter (a large, mostly idle grid would otherwise queue on it)
    if ((int)blockIdx.x >= tv.total[t]) return;
    int slot, rank;
    while (next_item(tv, t, &slot, &rank)) {
        const BatchInst &d = D[slot];
        DevState *st = S + slot;
        const int k = st->kcur;
        if (halted(st, k)) continue;
        MgsDev a;
        a.q = gfield<const TX>(d.q);
        a.V = gfield<const TV>(d.V);
        a.ldv = (size_t)d.ldv;
        a.k = k;
        a.L = d.L;
        a.hcol = gfield<double>(d.H) + (size_t)(k - 1) * d.ld;
        a.vout = gfield<TV>(d.V) + (size_t)k * d.ldv;
        a.cur = gfield<TX>(d.cur);
        a.partials = gfield<double>(d.mgs_part);
        a.rows = d.mgs_rows;
        a.st = st;
        a.bd_rel = d.bd_rel;
        a.step = k;
        a.ticket = nullptr;
        a.q64 = gfield<double>(d.q64);
        a.set_beta = 0;
        a.giv = GivensDev{};
        a.gram = nullptr;   // the engine runs the plain sweep
        if constexpr (E == 0) mgs_stream_body<TX, TV>(a, rank, d.mgs_G, lds);
        else mgs_body<TX, TV, E>(a, rank, d.mgs_G, lds);
    }
}

__global__ __launch_bounds__(64) void bgivens_kernel(const BatchInst *__restrict__ D, DevState *S, TabView tv)
{
    if ((int)blockIdx.x >= tv.nseg[kTGiv]) return;
    const int slot = tv.seg_slot(kTGiv, blockIdx.x);
    const BatchInst &d = D[slot];
    DevState *st = S + slot;
    const int k = st->kcur;
    if (halted(st, k)) return;
    double *rho = (d.method == ABG_METHOD_AB && d.need_res) ? gfield<double>(d.rho) : nullptr;
    if (k <= kWaveGivensMax)
        givens_wave(gfield<double>(d.H), d.ld, gfield<double>(d.R), gfield<double>(d.cs),
                    gfield<double>(d.sn), gfield<double>(d.g),
                    gfield<double>(d.Y) + (size_t)(k - 1) * d.k_max, rho, st->beta, k, st);
    else
        givens_step(gfield<double>(d.H), d.ld, gfield<double>(d.R), gfield<double>(d.cs),
                    gfield<double>(d.sn), gfield<double>(d.g),
                    gfield<double>(d.Y) + (size_t)(k - 1) * d.k_max, rho, st->beta, k, st);
}

// ||r_k|| by chunks: BA r = (b - A x0) - Z y_k, AB r = W_{k+1} rho. Each chunk's sum of
// squares is published; the last chunk to finish adds them in chunk order, writes the
// norm and raises the DP candidate stop.
template <typename TX, typename TV>
__global__ __launch_bounds__(kBlock) void bres_kernel(const BatchInst *__restrict__ D, DevState *S, TabView tv,
                                                      Tiles tl)
{
    __shared__ double cf[kMaxCoef];
    __shared__ double lds[kWaves];
    __shared__ int last;
    // uniform chunks: static round-robin
    for_each_item(tv, kTRes, 0, [&](int slot, int c) {
        const BatchInst &d = D[slot];
        DevState *st = S + slot;
        const int k = st->kcur;
        if (halted(st, k)) return;
        const bool ba = d.method == ABG_METHOD_BA;
        __syncthreads();   // the previous item's use of cf and `last` is done
        const int kk = ba ? k : k + 1;
        const double *coef =
            ba ? gfield<double>(d.Y) + (size_t)(k - 1) * d.k_max : gfield<double>(d.rho);
        for (int j = threadIdx.x; j < kk; j += kBlock) cf[j] = ba ? -coef[j] : coef[j];
        __syncthreads();
        const long long lo = (long long)c * d.chunk;
        const long long hi = min(lo + (long long)d.chunk, d.m);
        const TX *base = ba ? gfield<const TX>(d.rb0) : nullptr;
        double ss = 0.0;
        for (long long l0 = lo + threadIdx.x; l0 < hi; l0 += kResU * kBlock) {
            double acc[kResU];
            bool in[kResU];
#pragma unroll
            for (int u = 0; u < kResU; ++u) {
                const long long l = l0 + u * kBlock;
                in[u] = l < hi;
                acc[u] = (in[u] && base) ? to_f64(base[l]) : 0.0;
            }
            for (int j = 0; j < kk; ++j) {
                double x[kResU];
                if (ba) {
                    const TX *v = gfield<const TX>(d.Z) + (size_t)j * d.mp + l0;
#pragma unroll
                    for (int u = 0; u < kResU; ++u) x[u] = in[u] ? to_f64(v[u * kBlock]) : 0.0;
                } else {
                    const TV *v = gfield<const TV>(d.V) + (size_t)j * d.ldv + l0;
#pragma unroll
                    for (int u = 0; u < kResU; ++u) x[u] = in[u] ? to_f64(v[u * kBlock]) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < kResU; ++u) acc[u] = fma(cf[j], x[u], acc[u]);
            }
#pragma unroll
            for (int u = 0; u < kResU; ++u)
                if (in[u]) ss = fma(acc[u], acc[u], ss);
        }
        ss = block_sum(ss, lds);
        if (threadIdx.x == 0) {
            agent_store(d.part + c, ss);
            const unsigned prev = __hip_atomic_fetch_add(d.count, 1u, __ATOMIC_ACQ_REL,
                                                         __HIP_MEMORY_SCOPE_AGENT);
            last = prev == (unsigned)d.n_chunks - 1;
        }
        __syncthreads();
        if (!last) return;
        last_block_fence();
        double tsum = 0.0;
        for (int j = threadIdx.x; j < d.n_chunks; j += kBlock) tsum += agent_load(d.part + j);
        tsum = block_sum(tsum, lds);
        if (threadIdx.x == 0) {
            __hip_atomic_store(d.count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const double r = sqrt(tsum);
            st->res = r;
            if (!isfinite(r)) {
                st->error |= 2;
            } else if (st->dp_thr > 0.0 && r <= st->dp_thr && !st->stop) {
                st->stop = 1;
                st->stop_k = k;
                st->stop_reason = kStopDP;
            }
        }
    });
}

// ---- per-problem control kernels (launched by the host between rounds) ------------------
__global__ void activate_kernel(DevState *st)
{
    if (threadIdx.x != 0 || st->error) return;
    if (st->hnext == 0.0) {
        st->stop = 1;
        st->stop_k = 0;
        st->stop_reason = kStopZero;
        return;
    }
    st->beta = st->hnext;
    st->active = 1;
}

// After x_{stop_k} and lit = ||b - A x|| were formed for a DP candidate: accept, finish
// with `rej_status` (>= 0) if the problem cannot continue, or resume.
__global__ void confirm_kernel(DevState *st, double thr, int rej_status)
{
    if (threadIdx.x != 0) return;
    const double lit = st->lit;
    st->n_lit += 1;
    if (!isfinite(lit)) {
        st->status = ABG_ENAN;
    } else if (lit <= thr) {
        st->status = ABG_OK;
    } else if (rej_status >= 0) {
        st->status = rej_status;
    } else {
        st->stop = 0;
        st->stop_k = 0;
        st->stop_reason = kStopNone;
        return;
    }
    st->k_sel = st->stop_k;
    st->done = 1;
}

__global__ void final_kernel(DevState *st, int k_sel, int status)
{
    if (threadIdx.x != 0) return;
    st->status = isfinite(st->lit) ? status : ABG_ENAN;
    st->k_sel = k_sel;
    st->done = 1;
}

template <typename F> hipError_t capacity_of(F fn, int block, int *blocks)
{
    int dev = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, dev)) != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(fn),
                                                          block, 0)) != hipSuccess)
        return e;
    *blocks = std::max(1, per_cu) * prop.multiProcessorCount;
    return hipSuccess;
}

constexpr int kSnapRing = 4;

#define BCK(expr)                                   \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) return fail(ABG_EHIP); \
    } while (0)

// Stream callback after an engine round: returns the round's share of the Gram-Schmidt
// budget (touches only the budget object, no HIP call).
void release_round(void *budget) { static_cast<GroupBudget *>(budget)->release(GroupBudget::kUnits); }

}  // namespace

// ---- host engine ------------------------------------------------------------------------
struct Engine {
    enum Phase { kFree = 0, kRunning, kConfirming, kFinalizing };
    struct Slot {
        Phase phase = kFree;
        abg_request r{};
        const Geometry *g = nullptr;
        double thr = 0.0;
        int last_k = 0;
        int n_confirm = 0;
        int pend_k = 0;   // step whose iterate is being formed
        int gen = 0;
    };

    abg_precision p{};
    int max_slots = 0, device = 0;
    hipStream_t s = nullptr, cap_stream = nullptr;
    // second captured stream and the events that fork the AB chain onto it and join it
    hipStream_t cap_stream2 = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    BatchInst *d_desc = nullptr;
    DevState *d_st = nullptr;
    int *d_tab = nullptr;
    TabView tv{};
    BatchInst *h_desc = nullptr;     // pinned staging, one per slot
    DevState *h_init = nullptr;      // pinned staging, one per slot
    DevState *h_snap = nullptr;      // pinned ring of snapshots
    hipEvent_t ev[kSnapRing] = {};
    std::deque<int> inflight;
    int ring_next = 0;
    // the captured round, [0]: projector chains in sequence, [1]: as two branches
    hipGraph_t graph[2] = {};
    hipGraphExec_t exec[2] = {};
    bool dirty = true;
    Tiles tiles{0, 64, 2};
    int grid_proj = 0, grid_back = 0, grid_back64 = 0, grid_back_adj = 0, grid_back64_adj = 0;
    int grid_mgs_s = 0, grid_mgs_l = 0, grid_res = 0;
    hipEvent_t tev[2] = {};
    int cap_mgs_s = 0, cap_mgs_l = 0, cap_mgs_x = 0, grid_mgs_x = 0, cap_mgs_h = 0, grid_mgs_h = 0;
    int broken = 0;
    std::vector<Slot> slots;
    std::vector<std::pair<long long, int>> finished;
    long long rounds = 0;
    int gen_next = 0;

    int fail(int rc)
    {
        broken = rc;
        return rc;
    }

    ~Engine()
    {
        if (s) (void)hipStreamSynchronize(s);
        for (int v = 0; v < 2; ++v) {
            if (exec[v]) (void)hipGraphExecDestroy(exec[v]);
            if (graph[v]) (void)hipGraphDestroy(graph[v]);
        }
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
        for (auto &e : tev)
            if (e) (void)hipEventDestroy(e);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        if (cap_stream2) (void)hipStreamDestroy(cap_stream2);
        if (fork_ev) (void)hipEventDestroy(fork_ev);
        if (join_ev) (void)hipEventDestroy(join_ev);
        if (d_desc) (void)hipFree(d_desc);
        if (d_st) (void)hipFree(d_st);
        if (d_tab) (void)hipFree(d_tab);
        if (h_desc) (void)hipHostFree(h_desc);
        if (h_init) (void)hipHostFree(h_init);
        if (h_snap) (void)hipHostFree(h_snap);
    }

    template <typename TX, typename TV> hipError_t capacities()
    {
        hipError_t e;
        if ((e = capacity_of(bfwd_kernel<TX>, 256, &grid_proj)) != hipSuccess) return e;
        if ((e = capacity_of(bback_kernel<TX, 128, false>, kBackThreads, &grid_back)) != hipSuccess)
            return e;
        if ((e = capacity_of(bback_kernel<TX, 64, false>, kBackThreads, &grid_back64)) != hipSuccess)
            return e;
        if ((e = capacity_of(bback_kernel<TX, 128, true>, kBackThreads, &grid_back_adj)) != hipSuccess)
            return e;
        if ((e = capacity_of(bback_kernel<TX, 64, true>, kBackThreads, &grid_back64_adj)) != hipSuccess)
            return e;
        if ((e = capacity_of(bmgs_kernel<TX, TV, kMgsSmallE>, kBlock, &cap_mgs_s)) != hipSuccess) return e;
        if ((e = capacity_of(bmgs_kernel<TX, TV, kMgsLargeE>, kBlock, &cap_mgs_l)) != hipSuccess) return e;
        if ((e = capacity_of(bmgs_kernel<TX, TV, 0>, kBlock, &cap_mgs_x)) != hipSuccess) return e;
        if constexpr (sizeof(TV) < 8) {
            if ((e = capacity_of(bmgs_kernel<TX, TV, kMgsHugeE>, kBlock, &cap_mgs_h)) != hipSuccess)
                return e;
        } else {
            cap_mgs_h = 0;
        }
        grid_mgs_h = std::max(1, cap_mgs_h);
        grid_mgs_x = cap_mgs_x;
        if ((e = capacity_of(bres_kernel<TX, TV>, kBlock, &grid_res)) != hipSuccess) return e;
        grid_mgs_s = cap_mgs_s;
        grid_mgs_l = cap_mgs_l;
        grid_res = std::min(grid_res, 2048);
        return hipSuccess;
    }

    hipError_t caps_for_precision()
    {
        if (p.proj == ABG_F64) return capacities<double, double>();
        if (p.basis == ABG_F32) return capacities<float, float>();
        return capacities<float, bf16>();
    }

    // list t (interpolating back projector) and list t + 1 (its matched-pair twin)
    template <typename TX> void enqueue_back(hipStream_t q, const Tiles &tl, int t, int mode)
    {
        if (tl.ang_block == 64) {
            bback_kernel<TX, 64, false><<<grid_back64, kBackThreads, 0, q>>>(d_desc, d_st, tv, t, mode, tl);
            bback_kernel<TX, 64, true><<<grid_back64_adj, kBackThreads, 0, q>>>(d_desc, d_st, tv, t + 1,
                                                                                mode, tl);
        } else {
            bback_kernel<TX, 128, false><<<grid_back, kBackThreads, 0, q>>>(d_desc, d_st, tv, t, mode, tl);
            bback_kernel<TX, 128, true><<<grid_back_adj, kBackThreads, 0, q>>>(d_desc, d_st, tv, t + 1,
                                                                               mode, tl);
        }
    }

    // begin + the three projector phases (idempotent between rounds: they recompute the
    // round's z, t and q from w_k without advancing any problem). The BA chain (pad,
    // forward, back) and the AB chain (back, pad, forward) touch disjoint problems and
    // lists; with q2 the AB chain forks onto q2 and joins q after its last phase, so that
    // in a captured round the two chains are independent branches of the graph.
    template <typename TX> void enqueue_projectors_t(hipStream_t q, const Tiles &tl,
                                                     hipStream_t q2 = nullptr)
    {
        begin_kernel<<<kNumTab, 256, 0, q>>>(d_desc, d_st, tv, max_slots, tl);
        Tiles tf = tl;
        tf.stage = fwd_stage_eighths(p.proj);
        hipStream_t qa = q;
        if (q2) {
            (void)hipEventRecord(fork_ev, q);
            (void)hipStreamWaitEvent(q2, fork_ev, 0);
            qa = q2;
        }
        bpad_kernel<TX><<<grid_proj, 256, 0, q>>>(d_desc, d_st, tv, kTPadBA, 0, tl);
        enqueue_back<TX>(qa, tl, kTBackAB, 0);
        bfwd_kernel<TX><<<grid_proj, 256, 0, q>>>(d_desc, d_st, tv, kTFwdBA, 0, tf);
        bpad_kernel<TX><<<grid_proj, 256, 0, qa>>>(d_desc, d_st, tv, kTPadAB, 1, tl);
        enqueue_back<TX>(q, tl, kTBackBA, 1);
        bfwd_kernel<TX><<<grid_proj, 256, 0, qa>>>(d_desc, d_st, tv, kTFwdAB, 1, tf);
        if (q2) {
            (void)hipEventRecord(join_ev, q2);
            (void)hipStreamWaitEvent(q, join_ev, 0);
        }
    }

    void enqueue_projectors(hipStream_t q, const Tiles &tl)
    {
        if (p.proj == ABG_F64) enqueue_projectors_t<double>(q, tl);
        else enqueue_projectors_t<float>(q, tl);
    }

    template <typename TX, typename TV> void enqueue_round_t(hipStream_t q, hipStream_t q2)
    {
        enqueue_projectors_t<TX>(q, tiles, q2);
        bmgs_kernel<TX, TV, kMgsSmallE><<<grid_mgs_s, kBlock, 0, q>>>(d_desc, d_st, tv, kTMgsS);
        bmgs_kernel<TX, TV, kMgsLargeE><<<grid_mgs_l, kBlock, 0, q>>>(d_desc, d_st, tv, kTMgsL);
        if constexpr (sizeof(TV) < 8)
            bmgs_kernel<TX, TV, kMgsHugeE><<<grid_mgs_h, kBlock, 0, q>>>(d_desc, d_st, tv, kTMgsH);
        bmgs_kernel<TX, TV, 0><<<grid_mgs_x, kBlock, 0, q>>>(d_desc, d_st, tv, kTMgsX);
        bgivens_kernel<<<max_slots, 64, 0, q>>>(d_desc, d_st, tv);
        bres_kernel<TX, TV><<<grid_res, kBlock, 0, q>>>(d_desc, d_st, tv, tiles);
    }

    void enqueue_round(hipStream_t q, hipStream_t q2)
    {
        if (p.proj == ABG_F64) enqueue_round_t<double, double>(q, q2);
        else if (p.basis == ABG_F32) enqueue_round_t<float, float>(q, q2);
        else enqueue_round_t<float, bf16>(q, q2);
    }

    // Whether a round's AB chain runs beside its BA chain: it fills the tails of the
    // persistent projector kernels when the problems are small, but once one problem's
    // image and sinogram take a sizable share of the 256 MB Infinity Cache, the problems
    // of the two chains evict each other's data (measured: a mix with N <= 1024 5-9%
    // faster, the served stream with 2048^2 requests 2.5% slower).
    static constexpr double kForkMaxBytes = 32e6;
    bool fork_chains() const
    {
        double most = 0.0;
        const size_t es = dtype_size(p.proj);
        for (const auto &sl : slots)
            if (sl.phase != kFree && sl.g)
                most = std::max(most, (double)es * ((double)sl.g->N * sl.g->N + (double)sl.g->m()));
        return most < kForkMaxBytes;
    }

    // Drops both captured variants once the tiles changed; captures variant v if absent.
    int capture(int v)
    {
        if (dirty) {
            for (int u = 0; u < 2; ++u) {
                if (exec[u]) BCK(hipGraphExecDestroy(exec[u]));
                if (graph[u]) BCK(hipGraphDestroy(graph[u]));
                exec[u] = nullptr;
                graph[u] = nullptr;
            }
            dirty = false;
        }
        if (exec[v]) return ABG_OK;
        BCK(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
        enqueue_round(cap_stream, v ? cap_stream2 : nullptr);
        hipError_t le = hipGetLastError();
        hipGraph_t gr = nullptr;
        hipError_t ee = hipStreamEndCapture(cap_stream, &gr);
        if (le != hipSuccess || ee != hipSuccess) {
            if (gr) (void)hipGraphDestroy(gr);
            return fail(ABG_EHIP);
        }
        graph[v] = gr;
        BCK(hipGraphInstantiate(&exec[v], graph[v], nullptr, nullptr, 0));
        return ABG_OK;
    }

    int n_in(Phase ph) const
    {
        int c = 0;
        for (const auto &sl : slots) c += sl.phase == ph;
        return c;
    }
    int n_used() const { return (int)slots.size() - n_in(kFree); }

    int submit(const Geometry &g, const abg_request &r)
    {
        if (broken) return broken;
        int sidx = -1;
        for (int i = 0; i < max_slots; ++i)
            if (slots[i].phase == kFree) {
                sidx = i;
                break;
            }
        if (sidx < 0) return ABG_EFULL;
        // the back projector's window loads address the sinogram with 31-bit offsets
        if (!sinogram_fits_offset(g.m(), dtype_size(p.proj))) return ABG_EINVAL;
        const InstanceView v = instance_view(g, r.method, r.k_max, p, r.stop, r.ws);
        BatchInst d{};
        d.ang = g.dev;
        d.N = g.N;
        d.S = g.padded_stride();
        d.n_ang = g.n_ang;
        d.n_det = g.n_det;
        d.ds = g.ds;
        d.s0 = -0.5 * (g.n_det - 1) * g.ds;
        d.method = r.method;
        d.kind = r.bp_kind;
        d.k_max = r.k_max;
        d.ld = r.k_max + 1;
        d.L = v.L;
        d.ldv = v.ldv;
        d.mp = v.mp;
        d.n = g.n();
        d.m = g.m();
        d.V = v.V;
        d.Z = v.Z;
        d.cur = v.cur;
        d.q = v.q;
        d.rb0 = v.rb0;
        d.tm = v.tm;
        d.tn = v.tn;
        d.xr = v.fpws;
        d.xc = static_cast<char *>(v.fpws) + (size_t)g.N * g.padded_stride() * dtype_size(p.proj);
        d.H = v.H;
        d.R = v.R;
        d.cs = v.cs;
        d.sn = v.sn;
        d.g = v.g;
        d.Y = v.Y;
        d.rho = v.rho;
        d.part = v.part;
        d.mgs_part = v.mgs_part;
        d.q64 = v.q64;
        d.mgs_rows = v.mgs_rows;
        d.count = v.count;
        d.bd_rel = (p.basis == ABG_F64 && p.proj == ABG_F64) ? 1e-14 : 1e-6;
        d.need_res = r.stop.kind == ABG_STOP_DP;
        d.fwd_rays = 256 >> fwd_lg_angles_per_block(g);
        // Gram-Schmidt class: the smallest register tile whose block group the device
        // holds at once (the small tile while its group stays small), else the streaming
        // variant. A group must be resident as a whole: its size stays within the
        // kernel's resident-block capacity.
        auto groups = [&](int E) {
            return (v.L + (long long)kBlock * E - 1) / ((long long)kBlock * E);
        };
        long long G = groups(kMgsSmallE);
        d.mgs_class = 0;
        int capG = cap_mgs_s;
        if (G > kMgsSmallMaxG) {
            G = groups(kMgsLargeE);
            d.mgs_class = 1;
            capG = cap_mgs_l;
            if (G > cap_mgs_l && cap_mgs_h > 0 && groups(kMgsHugeE) <= cap_mgs_h) {
                G = groups(kMgsHugeE);
                d.mgs_class = 3;
                capG = cap_mgs_h;
            }
            if (G > capG) {
                if (!v.q64) return ABG_EINVAL;
                d.mgs_class = 2;
                G = kMgsStreamG;
                capG = cap_mgs_x;
            }
        }
        if (G > capG || 2LL * v.mgs_rows * G > v.mgs_part_cap) return ABG_EINVAL;
        d.mgs_G = (int)std::max(1LL, G);
        long long chunk = 8192;
        while ((d.m + chunk - 1) / chunk > v.part_cap) chunk *= 2;
        d.chunk = (int)chunk;
        d.n_chunks = (int)((d.m + chunk - 1) / chunk);

        Slot &sl = slots[sidx];
        sl = Slot{};
        sl.r = r;
        sl.g = &g;
        sl.thr = r.stop.kind == ABG_STOP_DP ? r.stop.tau * r.stop.noise_norm : 0.0;
        const double slack = p.basis == ABG_F64 ? 1e-6 : (p.basis == ABG_F32 ? 1e-3 : 5e-2);
        sl.gen = ++gen_next;
        DevState init{};
        init.gen = sl.gen;
        init.dp_thr = r.stop.kind == ABG_STOP_DP ? sl.thr * (1.0 + slack) : 0.0;
        h_desc[sidx] = d;
        h_init[sidx] = init;
        BCK(hipMemcpyAsync(d_desc + sidx, h_desc + sidx, sizeof(BatchInst), hipMemcpyHostToDevice, s));
        BCK(hipMemcpyAsync(d_st + sidx, h_init + sidx, sizeof(DevState), hipMemcpyHostToDevice, s));
        int rc = instance_init(g, r.method, r.bp_kind, r.k_max, r.stop, p, r.ws, r.b, r.x0,
                               d_st + sidx, s);
        if (rc != ABG_OK) return fail(rc);
        activate_kernel<<<1, 64, 0, s>>>(d_st + sidx);
        BCK(hipGetLastError());
        sl.phase = kRunning;
        if (r.info) {
            r.info->k_stop = r.info->k_done = r.info->n_literal = 0;
            r.info->status = ABG_OK;
        }
        return ABG_OK;
    }

    // Average time of the projector phases of one round with tile shape tl, over `reps`
    // repetitions on the current problems (0 when none is running).
    int time_projectors(const Tiles &tl, int reps, double *ms)
    {
        *ms = 0.0;
        if (n_in(kRunning) == 0) return ABG_OK;
        for (auto &e : tev)
            if (!e) BCK(hipEventCreate(&e));
        enqueue_projectors(s, tl);   // warm-up
        BCK(hipGetLastError());
        BCK(hipEventRecord(tev[0], s));
        for (int r = 0; r < reps; ++r) enqueue_projectors(s, tl);
        BCK(hipGetLastError());
        BCK(hipEventRecord(tev[1], s));
        BCK(hipEventSynchronize(tev[1]));
        float t = 0.f;
        BCK(hipEventElapsedTime(&t, tev[0], tev[1]));
        *ms = (double)t / std::max(1, reps);
        return ABG_OK;
    }

    // Times every tile shape on the current problems and keeps the fastest.
    int autotune(int reps, Tiles *best_out, double *best_ms)
    {
        if (broken) return broken;
        if ((int)inflight.size() > 0) {
            int rc = drain();
            if (rc) return rc;
        }
        Tiles best = tiles;
        double bms = INFINITY;
        for (int rays : {0, 64, 128, 256})
            for (int ab : {64, 128})
            for (int sc : {0, 1, 2}) {
                const Tiles tl{rays, ab, sc};
                double ms = 0.0;
                int rc = time_projectors(tl, reps, &ms);
                if (rc) return rc;
                if (ms > 0.0 && ms < bms) {
                    bms = ms;
                    best = tl;
                }
            }
        if (best.rays != tiles.rays || best.ang_block != tiles.ang_block ||
            best.sched != tiles.sched) {
            tiles = best;
            dirty = true;
        }
        *best_out = tiles;
        *best_ms = std::isfinite(bms) ? bms : 0.0;
        return ABG_OK;
    }

    // x_k and ||b - A x_k|| for the problem in slot i
    int form_x(int i, int k)
    {
        Slot &sl = slots[i];
        const abg_request &r = sl.r;
        DevState *st = d_st + i;
        int rc = instance_form_x(*sl.g, r.method, r.bp_kind, r.k_max, r.stop, p, r.ws, k, r.b,
                                 r.x0, r.x, st, &st->lit, s);
        if (rc != ABG_OK) return fail(rc);
        sl.pend_k = k;
        return ABG_OK;
    }

    void finish(int i, const DevState &h, int status)
    {
        Slot &sl = slots[i];
        abg_info *info = sl.r.info;
        if (info) {
            info->k_stop = h.k_sel;
            info->k_done = h.k;
            info->status = status;
            info->n_literal = h.n_lit;
            info->res_norm = h.lit;
            info->ncp_dist = 0.0;
            info->beta = h.beta;
        }
        finished.emplace_back(sl.r.tag, status);
        sl.phase = kFree;
    }

    // Host side of one snapshot of every problem's scalars.
    int process(const DevState *snap)
    {
        for (int i = 0; i < max_slots; ++i) {
            Slot &sl = slots[i];
            if (sl.phase == kFree) continue;
            const DevState &h = snap[i];
            if (h.gen != sl.gen) continue;   // copy taken before this admission
            abg_info *info = sl.r.info;
            if (h.k > sl.last_k) {
                // a round advances a problem by at most one step
                if (info && info->ls_hist && h.k - 1 < info->hist_len) info->ls_hist[h.k - 1] = h.ls;
                if (info && info->res_hist && h.k - 1 < info->hist_len &&
                    sl.r.stop.kind == ABG_STOP_DP)
                    info->res_hist[h.k - 1] = h.res;
                sl.last_k = h.k;
            }
            if (h.error) {
                DevState hh = h;
                hh.k_sel = 0;
                finish(i, hh, (h.error & 1) ? ABG_EDEVICE : ABG_ENAN);
                continue;
            }
            if (h.done) {
                if (sl.phase == kConfirming && info && info->res_hist && h.k_sel - 1 >= 0 &&
                    h.k_sel - 1 < info->hist_len)
                    info->res_hist[h.k_sel - 1] = h.lit;
                finish(i, h, h.status);
                continue;
            }
            if (sl.phase == kConfirming) {
                if (h.n_lit >= sl.n_confirm) {
                    // rejected: the problem runs again
                    if (info && info->res_hist && sl.pend_k - 1 < info->hist_len)
                        info->res_hist[sl.pend_k - 1] = h.lit;
                    sl.phase = kRunning;
                }
                continue;
            }
            if (sl.phase != kRunning) continue;
            if (h.stop && h.stop_reason == kStopZero) {
                int rc = form_x(i, 0);
                if (rc) return rc;
                final_kernel<<<1, 64, 0, s>>>(d_st + i, 0, ABG_ZERO_RHS);
                BCK(hipGetLastError());
                sl.phase = kFinalizing;
            } else if (h.stop && h.stop_reason == kStopDP && h.stop_k == h.k && h.k > 0) {
                int rc = form_x(i, h.k);
                if (rc) return rc;
                int rej = -1;
                if (h.bd_k == h.k) rej = ABG_BREAKDOWN;
                else if (h.k >= sl.r.k_max) rej = ABG_NOT_CONVERGED;
                confirm_kernel<<<1, 64, 0, s>>>(d_st + i, sl.thr, rej);
                BCK(hipGetLastError());
                ++sl.n_confirm;
                sl.phase = kConfirming;
            } else if (h.k > 0 && h.bd_k == h.k) {
                int rc = form_x(i, h.k);
                if (rc) return rc;
                final_kernel<<<1, 64, 0, s>>>(d_st + i, h.k, ABG_BREAKDOWN);
                BCK(hipGetLastError());
                sl.phase = kFinalizing;
            } else if (h.k >= sl.r.k_max) {
                int rc = form_x(i, h.k);
                if (rc) return rc;
                const int status = sl.r.stop.kind == ABG_STOP_DP ? ABG_NOT_CONVERGED : ABG_OK;
                final_kernel<<<1, 64, 0, s>>>(d_st + i, h.k, status);
                BCK(hipGetLastError());
                sl.phase = kFinalizing;
            }
        }
        return ABG_OK;
    }

    int wait_oldest()
    {
        const int r = inflight.front();
        inflight.pop_front();
        BCK(hipEventSynchronize(ev[r]));
        return process(h_snap + (size_t)r * max_slots);
    }

    // One round: replay the graph (if a problem is running), copy the scalars, and
    // process the previous round's copy.
    int step()
    {
        if (broken) return broken;
        if (n_used() == 0 && inflight.empty()) return ABG_OK;
        if ((int)inflight.size() >= 2) {
            int rc = wait_oldest();
            if (rc) return rc;
        }
        if (n_in(kRunning) > 0) {
            const int v = fork_chains() ? 1 : 0;
            if (dirty || !exec[v]) {
                int rc = capture(v);
                if (rc) return rc;
            }
            // the round's Gram-Schmidt grids take what the device holds: the whole
            // budget, returned by a stream callback once the round has run
            GroupBudget &budget = device_group_budget();
            budget.acquire(GroupBudget::kUnits);
            hipError_t e = hipGraphLaunch(exec[v], s);
            if (e == hipSuccess) e = hipLaunchHostFunc(s, release_round, &budget);
            if (e != hipSuccess) {
                (void)hipStreamSynchronize(s);
                budget.release(GroupBudget::kUnits);
                return fail(ABG_EHIP);
            }
            ++rounds;
        }
        const int r = ring_next;
        ring_next = (ring_next + 1) % kSnapRing;
        BCK(hipMemcpyAsync(h_snap + (size_t)r * max_slots, d_st, sizeof(DevState) * max_slots,
                           hipMemcpyDeviceToHost, s));
        BCK(hipEventRecord(ev[r], s));
        inflight.push_back(r);
        return ABG_OK;
    }

    int drain()
    {
        while (!inflight.empty()) {
            int rc = wait_oldest();
            if (rc) return rc;
        }
        return ABG_OK;
    }
};

int engine_create(abg_precision p, int max_slots, hipStream_t s, Engine **out)
{
    const bool ok = (p.proj == ABG_F64 && p.basis == ABG_F64) ||
                    (p.proj == ABG_F32 && (p.basis == ABG_F32 || p.basis == ABG_BF16));
    if (!ok || max_slots < 1 || max_slots > 4096) return ABG_EINVAL;
    Engine *e = new (std::nothrow) Engine();
    if (!e) return ABG_EHIP;
    e->p = p;
    e->max_slots = max_slots;
    e->s = s;
    e->slots.resize(max_slots);
    auto bad = [&]() {
        delete e;
        return ABG_EHIP;
    };
    if (hipGetDevice(&e->device) != hipSuccess) return bad();
    if (hipStreamCreateWithFlags(&e->cap_stream, hipStreamNonBlocking) != hipSuccess) return bad();
    if (hipStreamCreateWithFlags(&e->cap_stream2, hipStreamNonBlocking) != hipSuccess) return bad();
    if (hipEventCreateWithFlags(&e->fork_ev, hipEventDisableTiming) != hipSuccess) return bad();
    if (hipEventCreateWithFlags(&e->join_ev, hipEventDisableTiming) != hipSuccess) return bad();
    const size_t tab_ints = (2 + kRanges) * kNumTab + 2 * (size_t)kNumTab * max_slots;
    if (hipMalloc(&e->d_desc, sizeof(BatchInst) * max_slots) != hipSuccess) return bad();
    if (hipMalloc(&e->d_st, sizeof(DevState) * max_slots) != hipSuccess) return bad();
    if (hipMalloc(&e->d_tab, sizeof(int) * tab_ints) != hipSuccess) return bad();
    if (hipHostMalloc((void **)&e->h_desc, sizeof(BatchInst) * max_slots, hipHostMallocDefault) != hipSuccess) return bad();
    if (hipHostMalloc((void **)&e->h_init, sizeof(DevState) * max_slots, hipHostMallocDefault) != hipSuccess) return bad();
    if (hipHostMalloc((void **)&e->h_snap, sizeof(DevState) * max_slots * kSnapRing, hipHostMallocDefault) != hipSuccess) return bad();
    for (auto &ev : e->ev)
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return bad();
    e->tv.nseg = e->d_tab;
    e->tv.total = e->d_tab + kNumTab;
    e->tv.ticket = reinterpret_cast<unsigned *>(e->d_tab + 2 * kNumTab);
    e->tv.slot = e->d_tab + (2 + kRanges) * kNumTab;
    e->tv.first = e->tv.slot + (size_t)kNumTab * max_slots;
    e->tv.max_slots = max_slots;
    // every slot starts idle: zero scalars and descriptors
    if (launch_fill_u32(reinterpret_cast<unsigned *>(e->d_st), sizeof(DevState) * max_slots / 4, 0u, s) != hipSuccess) return bad();
    if (launch_fill_u32(reinterpret_cast<unsigned *>(e->d_desc), sizeof(BatchInst) * max_slots / 4, 0u, s) != hipSuccess) return bad();
    if (launch_fill_u32(reinterpret_cast<unsigned *>(e->d_tab), tab_ints, 0u, s) != hipSuccess) return bad();
    if (e->caps_for_precision() != hipSuccess) return bad();
    *out = e;
    return ABG_OK;
}

void engine_destroy(Engine *e) { delete e; }

int engine_submit(Engine *e, const Geometry &g, const abg_request &r) { return e->submit(g, r); }

int engine_step(Engine *e, int *n_running)
{
    const int rc = e->step();
    if (n_running) *n_running = e->n_used();
    return rc;
}

int engine_poll(Engine *e, long long *tags, int *status, int max, int *n)
{
    int c = 0;
    while (c < max && c < (int)e->finished.size()) {
        if (tags) tags[c] = e->finished[c].first;
        if (status) status[c] = e->finished[c].second;
        ++c;
    }
    e->finished.erase(e->finished.begin(), e->finished.begin() + c);
    *n = c;
    return e->broken ? e->broken : ABG_OK;
}

int engine_pending(const Engine *e) { return e->n_used() + (int)e->finished.size(); }

int engine_set_tiles(Engine *e, int rays, int ang_block, int sched)
{
    if (rays != 0 && rays != 64 && rays != 128 && rays != 256) return ABG_EINVAL;
    if (ang_block != 64 && ang_block != 128) return ABG_EINVAL;
    if (sched < 0 || sched > 2) return ABG_EINVAL;
    if (e->tiles.rays != rays || e->tiles.ang_block != ang_block || e->tiles.sched != sched) {
        e->tiles = Tiles{rays, ang_block, sched};
        e->dirty = true;
    }
    return ABG_OK;
}

int engine_get_tiles(const Engine *e, int *rays, int *ang_block, int *sched)
{
    *rays = e->tiles.rays;
    *ang_block = e->tiles.ang_block;
    *sched = e->tiles.sched;
    return ABG_OK;
}

int engine_autotune(Engine *e, int reps, int *rays, int *ang_block, int *sched, double *ms)
{
    Tiles t{};
    const int rc = e->autotune(reps, &t, ms);
    *rays = t.rays;
    *ang_block = t.ang_block;
    *sched = t.sched;
    return rc;
}

int engine_device(const Engine *e) { return e->device; }
hipStream_t engine_stream(const Engine *e) { return e->s; }
int engine_precision(const Engine *e, abg_precision *p)
{
    *p = e->p;
    return ABG_OK;
}
long long engine_rounds(const Engine *e) { return e->rounds; }

}  // namespace abg
