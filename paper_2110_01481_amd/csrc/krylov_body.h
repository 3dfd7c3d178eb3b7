// Device helpers of the Krylov kernels (conversions, fixed-order reductions, device-scope
// publication of partial sums, the Givens update), shared by the single-problem kernels
// (krylov.hip) and the batched kernels (batch.hip).
#pragma once

#include <cmath>

#include "abg_internal.h"

namespace abg {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr unsigned kSpinLimit = 1u << 22;
constexpr int kGatherRows = 8;    // slot rows polled together by gather_rows
constexpr int kMaxCoef = 512;

// ---- element access ------------------------------------------------------------------
__device__ inline double to_f64(double v) { return v; }
__device__ inline double to_f64(float v) { return (double)v; }
__device__ inline double to_f64(bf16 v) { return (double)__uint_as_float((unsigned)v.bits << 16); }

template <typename T> __device__ inline T from_f64(double v);
template <> __device__ inline double from_f64<double>(double v) { return v; }
template <> __device__ inline float from_f64<float>(double v) { return (float)v; }
template <> __device__ inline bf16 from_f64<bf16>(double v)
{
    // round to float, then to the nearest bf16 (ties to even); NaN stays NaN
    const unsigned u = __float_as_uint((float)v);
    bf16 r;
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
        r.bits = (uint16_t)((u >> 16) | 0x40u);
    } else {
        const unsigned lsb = (u >> 16) & 1u;
        r.bits = (uint16_t)((u + 0x7fffu + lsb) >> 16);
    }
    return r;
}
template <typename T> __device__ inline T zero_of();
template <> __device__ inline double zero_of<double>() { return 0.0; }
template <> __device__ inline float zero_of<float>() { return 0.0f; }
template <> __device__ inline bf16 zero_of<bf16>() { return bf16{0}; }

// ---- reductions ----------------------------------------------------------------------
// Value of a double held by lane l (a compile-time lane) of the wave.
__device__ inline double readlane_first(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Butterfly sum: lanes l and l^d add the same two operands, so every lane ends with the
// same value regardless of position.
__device__ inline double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Wave sum through DPP moves only (no LDS permutes), the same value in every lane: within
// each row of 16 lanes x += ror(x, 8), x += ror(x, 4), then the quad swaps of 2 and 1
// (each add takes the same two operands in the lanes it pairs, so the row's lanes agree);
// the four row totals are then added in row order from lanes 0, 16, 32, 48.
template <int CTRL> __device__ inline double dpp_move(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline double wave_sum_dpp(double v)
{
    v += dpp_move<0x128>(v);   // row_ror:8
    v += dpp_move<0x124>(v);   // row_ror:4
    v += dpp_move<0x4e>(v);    // quad_perm [2,3,0,1]
    v += dpp_move<0xb1>(v);    // quad_perm [1,0,3,2]
    return ((readlane_first(v, 0) + readlane_first(v, 16)) + readlane_first(v, 32)) +
           readlane_first(v, 48);
}

// Block sum returned to every thread, fixed order.
__device__ inline double block_sum(double v, double *lds)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) s += lds[i];
    return s;
}

__device__ inline double agent_load(const double *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Publishes a partial sum at device scope and waits until the write has been performed
// (the exchange's returned value is consumed). The counter increment after it is an
// agent-scope acquire-release, which orders the store before it in the memory model as
// well; partials are read back only with device-scope atomic loads, after an
// agent-scope acquire fence in the block that read the last count (last_block_fence).
__device__ inline void agent_store(double *p, double v)
{
    const double old = __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    asm volatile("" ::"v"(old) : "memory");
}

// In the last block of a counted reduction, after the barrier that shares the count:
// every thread's later loads see what the other blocks wrote before their increments.
__device__ inline void last_block_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// ---- group reductions through value slots -----------------------------------------------
// A block group reduces a scalar by writing one partial per block into a slot that holds
// kSlotEmpty beforehand; readers poll the slots until none is empty. The value is its own
// arrival signal, so a reduction costs one store and one round of polling, with no
// counter and no ordering between different addresses. kSlotEmpty is a signalling NaN,
// which arithmetic never produces (NaN partials are stored as the default quiet NaN).
constexpr unsigned long long kSlotEmpty = 0x7ff4dead0000c0deull;

__device__ inline void publish(double *slot, double v)
{
    if (v != v) v = __longlong_as_double(0x7ff8000000000000ll);
    __hip_atomic_store(slot, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of the G published partials, the same in every block and every thread (thread t
// adds slots t, t + kBlock, ... in order, then the fixed-order block sum). The wait is
// bounded: on timeout the sticky error flag is raised; a raised flag ends every wait.
__device__ inline double gather_total(const double *slots, int G, double *lds, int *err)
{
    double s = 0.0;
    unsigned spins = 0;
    bool quit = false;
    for (int j0 = 0; j0 < G && !quit; j0 += kBlock) {
        const int j = j0 + (int)threadIdx.x;
        double v = 0.0;
        int have = j >= G;
        for (;;) {
            if (!have) {
                v = agent_load(slots + j);
                have = (unsigned long long)__double_as_longlong(v) != kSlotEmpty;
            }
            if (__syncthreads_and(have)) break;
            ++spins;
            if ((spins & 255u) == 0) {
                const int e = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (spins > kSpinLimit && threadIdx.x == 0 && !e)
                    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (__syncthreads_or(e != 0 || spins > kSpinLimit)) {
                    quit = true;
                    break;
                }
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (j < G) s += v;
    }
    return block_sum(s, lds);
}

// Totals of slot rows 0..R-1 (each over the G published partials) into tot[0..R-1], the
// same in every block. Groups of at most kBlock blocks: thread t reads column t of
// kGatherRows rows at once, so the rows of one exchange cost one round of polling
// together; the waves' sums are added in wave order. Larger groups: gather_total row by
// row. Bounded wait as gather_total.
__device__ inline void gather_rows(const double *tab, int G, int R, double (*red)[kGatherRows],
                                   double *tot, double *lds, int *err)
{
    if (G > kBlock) {
        for (int r = 0; r < R; ++r) {
            const double t = gather_total(tab + (size_t)r * G, G, lds, err);
            if (threadIdx.x == 0) tot[r] = t;
        }
        __syncthreads();
        return;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = threadIdx.x;
    const int jc = min(j, G - 1);
    unsigned spins = 0;
    bool quit = false;
    for (int c0 = 0; c0 < R; c0 += kGatherRows) {
        const int nr = min(kGatherRows, R - c0);
        const double *col = tab + (size_t)c0 * G + jc;
        double v[kGatherRows];
        // every load issued before any is tested (rows past nr re-read row nr - 1)
#pragma unroll
        for (int r = 0; r < kGatherRows; ++r) v[r] = agent_load(col + (size_t)min(r, nr - 1) * G);
        unsigned need = 0;
#pragma unroll
        for (int r = 0; r < kGatherRows; ++r)
            if ((unsigned long long)__double_as_longlong(v[r]) == kSlotEmpty) need |= 1u << r;
        if (j >= G) need = 0;
        while (!quit && !__syncthreads_and(need == 0)) {
            ++spins;
            if ((spins & 255u) == 0) {
                const int e = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (spins > kSpinLimit && threadIdx.x == 0 && !e)
                    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (__syncthreads_or(e != 0 || spins > kSpinLimit)) {
                    quit = true;
                    break;
                }
            }
            __builtin_amdgcn_s_sleep(1);
            if (need) {
#pragma unroll
                for (int r = 0; r < kGatherRows; ++r) {
                    v[r] = agent_load(col + (size_t)min(r, nr - 1) * G);
                    if ((unsigned long long)__double_as_longlong(v[r]) != kSlotEmpty)
                        need &= ~(1u << r);
                }
            }
        }
        // all kGatherRows wave sums in one straight-line block (rows past nr dropped)
#pragma unroll
        for (int r = 0; r < kGatherRows; ++r) v[r] = wave_sum_dpp(j < G ? v[r] : 0.0);
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r < kGatherRows; ++r)
                if (r < nr) red[wave][r] = v[r];
        }
        __syncthreads();
        if ((int)threadIdx.x < nr) {
            double t = red[0][threadIdx.x];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) t += red[w][threadIdx.x];
            tot[c0 + threadIdx.x] = t;
        }
        __syncthreads();
    }
}

// ---- modified Gram-Schmidt ------------------------------------------------------------
// One Arnoldi step's orthogonalisation of q_k against w_1..w_k by G blocks (ranks
// 0..G-1): q_k stays in FP64 registers (E elements per thread), each basis vector is read
// once, and every inner product is one group reduction in a fixed order. Writes
// h_{1,k}..h_{k+1,k}, w_{k+1} (basis dtype) and its copy in q's dtype.
//
// Reduction slots: two tables (step parity) of `rows` rows x G doubles; step k uses
// table k & 1, row i for <q, w_i>, row k for ||q||^2 after the sweep and row k + 1 for
// ||q_k||^2 before it. Each rank clears its own column of the other table (rows up to
// k + 2) for the next step; both tables start cleared.
// The Givens update that follows Gram-Schmidt step k, done by the block of rank 0 once
// h_{1..k+1,k} are known (H null: none).
struct GivensDev {
    double *H, *R, *cs, *sn, *g, *y, *rho;
    int ld;
    DevState *snap;     // host-visible copy of the scalars after the update (or null)
};

struct MgsDev {
    const void *q;
    const void *V;
    size_t ldv;
    int k;
    long long L;
    double *hcol;
    void *vout;
    void *cur;
    double *partials;
    int rows;
    unsigned *ticket;
    DevState *st;
    double bd_rel;
    int step;
    double *q64;       // FP64 scratch of the streaming variant (vectors longer than kRegMaxL)
    int set_beta;      // step 0 of a single solve: beta = ||r_0||, or the zero-rhs stop
    GivensDev giv;
    // strictly lower triangle of the basis Gram matrix, row i (<w_i, w_j>, j < i) packed
    // from i(i-1)/2; null: every step runs the plain sweep
    double *gram;
};

// ---- low-synchronisation Gram-Schmidt (inverse compact WY form of MGS) ------------------
// MGS's coefficients h_i = <q - sum_{j<i} h_j w_j, w_i> equal, in exact arithmetic, the
// forward substitution h_i = <q, w_i> - sum_{j<i} <w_i, w_j> h_j. Steps 2 <= k <=
// kIcwyMaxK therefore exchange the k inner products <q, w_i>, ||q_k||^2 and the new Gram
// row <w_k, w_j> (j < k) in one group reduction, solve for h in FP64 (every block alike),
// subtract sum_i h_i w_i in MGS's order and exchange ||q||^2 in a second reduction: two
// reductions per step instead of k + 1. Slot rows of step k: <q, w_i> in 0..k-1,
// ||q_k||^2 in k, the Gram row in k+1..2k-1, ||q||^2 after the update in 2k.
struct IcwyLds {
    double part[kWaves][2 * kIcwyMaxK];                   // wave partials of rows 0..2k-1
    double tot[2 * kIcwyMaxK];                            // group totals of rows 0..2k-1
    double red[kWaves][kGatherRows];
    double tri[kIcwyMaxK * (kIcwyMaxK - 1) / 2];          // Gram rows 0..k-2, packed
    double h[kIcwyMaxK];
};

// One block of NT threads. Column k-1 of H has just been written by mgs; R holds the
// rotated columns,
// cs/sn the rotations, g the rotated right-hand side. Writes y_k (k entries) and, when
// rho is given, rho = beta e_1 - H_k y_k.
template <int NT = 64>
__device__ inline void givens_step(double *H, int ld, double *R, double *cs, double *sn,
                                   double *g, double *y, double *rho, double beta, int k,
                                   DevState *st)
{
    __shared__ double gg[kMaxCoef];
    __shared__ double ys[kMaxCoef];
    const int lane = threadIdx.x;
    const int j = k - 1;
    double *Hc = H + (size_t)j * ld;
    double *Rc = R + (size_t)j * ld;
    const bool bd = st->bd_k == k;
    for (int i = lane; i <= k; i += NT) Rc[i] = (i == k && bd) ? 0.0 : Hc[i];
    __syncthreads();
    if (lane == 0) {
        for (int i = 0; i < j; ++i) {
            const double a = Rc[i], b = Rc[i + 1];
            Rc[i] = cs[i] * a + sn[i] * b;
            Rc[i + 1] = -sn[i] * a + cs[i] * b;
        }
        const double a = Rc[j], b = Rc[k];
        const double r = hypot(a, b);
        double c = 1.0, s = 0.0;
        if (r > 0.0) {
            c = a / r;
            s = b / r;
        } else {
            st->error |= 4;
        }
        cs[j] = c;
        sn[j] = s;
        Rc[j] = r;
        Rc[k] = 0.0;
        const double gj = g[j];
        g[j] = c * gj;
        g[k] = -s * gj;
        st->ls = fabs(g[k]);
        st->k = k;
    }
    __syncthreads();
    for (int i = lane; i < k; i += NT) gg[i] = g[i];
    __syncthreads();
    for (int jj = k - 1; jj >= 0; --jj) {
        const double yj = gg[jj] / R[(size_t)jj * ld + jj];
        if (lane == 0) ys[jj] = yj;
        for (int i = lane; i < jj; i += NT) gg[i] -= R[(size_t)jj * ld + i] * yj;
        __syncthreads();
    }
    for (int i = lane; i < k; i += NT) y[i] = ys[i];
    if (rho) {
        for (int i = lane; i <= k; i += NT) {
            double acc = (i == 0) ? beta : 0.0;
            for (int jj = (i > 0 ? i - 1 : 0); jj < k; ++jj) acc -= H[(size_t)jj * ld + i] * ys[jj];
            rho[i] = acc;
        }
    }
}

// Value of a double held by lane l of the wave (l uniform).
__device__ inline double readlane_d(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Largest step that givens_wave takes (rows 0..k of the new column, one per lane).
constexpr int kWaveGivensMax = 63;

// givens_step for k <= kWaveGivensMax by the first wave of the block (lanes 0..63): the
// new column, the previous rotations and g are held one entry per lane and scalars move
// between lanes by readlane, so the sequential parts (applying the rotations, the back
// substitution) run from registers; the columns of R are fetched eight at a time. Same
// arithmetic, in the same order, as givens_step. Lane 0 writes the scalars.
__device__ inline void givens_wave(double *H, int ld, double *R, double *cs, double *sn,
                                   double *g, double *y, double *rho, double beta, int k,
                                   DevState *st)
{
    const int lane = threadIdx.x & 63;
    const int j = k - 1;
    const double *Hc = H + (size_t)j * ld;
    double *Rc = R + (size_t)j * ld;
    const bool bd = st->bd_k == k;
    const double hv = lane <= k ? ((lane == k && bd) ? 0.0 : Hc[lane]) : 0.0;
    const double cv = lane < j ? cs[lane] : 0.0;
    const double sv = lane < j ? sn[lane] : 0.0;
    double gl = lane < k ? g[lane] : 0.0;
    // rotations 0..j-1 applied to the column: t carries entry i+1 down the column
    double t = readlane_d(hv, 0);
    double rv = 0.0;   // this lane's entry of the rotated column
    for (int i = 0; i < j; ++i) {
        const double a = t, b = readlane_d(hv, i + 1);
        const double ci = readlane_d(cv, i), si = readlane_d(sv, i);
        const double o = ci * a + si * b;
        t = -si * a + ci * b;
        if (lane == i) rv = o;
    }
    const double a = t, b = readlane_d(hv, k);
    const double r = hypot(a, b);
    double c = 1.0, s = 0.0;
    if (r > 0.0) {
        c = a / r;
        s = b / r;
    } else if (lane == 0) {
        st->error |= 4;
    }
    if (lane == j) rv = r;
    if (lane < k) Rc[lane] = rv;
    if (lane == k) Rc[k] = 0.0;
    const double gj = readlane_d(gl, j);
    if (lane == 0) {
        cs[j] = c;
        sn[j] = s;
        g[j] = c * gj;
        g[k] = -s * gj;
        st->ls = fabs(-s * gj);
        st->k = k;
    }
    if (lane == j) gl = c * gj;
    // back substitution R_k y = g[0..k), column by column from the last
    double yv = 0.0;   // y[lane]
    for (int jb = j; jb >= 0; jb -= 8) {
        double col[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int jj = jb - u;
            col[u] = jj < 0 ? 0.0 : (jj == j ? rv : (lane <= jj ? R[(size_t)jj * ld + lane] : 0.0));
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int jj = jb - u;
            if (jj < 0) break;
            const double yj = readlane_d(gl, jj) / readlane_d(col[u], jj);
            if (lane == jj) yv = yj;
            if (lane < jj) gl -= col[u] * yj;
        }
    }
    if (lane < k) y[lane] = yv;
    if (rho) {
        double acc = lane == 0 ? beta : 0.0;
        for (int jj = 0; jj < k; ++jj) {
            const double yj = readlane_d(yv, jj);
            if (lane <= k && jj >= lane - 1) acc -= H[(size_t)jj * ld + lane] * yj;
        }
        if (lane <= k) rho[lane] = acc;
    }
}

// Entry idx (uniform) of a vector held NE entries per lane (entry e*64 + lane in v[e]).
template <int NE>
__device__ inline double readlane_n(const double (&v)[NE], int idx)
{
    double x = 0.0;
#pragma unroll
    for (int e = 0; e < NE; ++e)
        if ((idx >> 6) == e) x = readlane_d(v[e], idx & 63);
    return x;
}

// Largest step that givens_wave2 takes (rows 0..k of the new column, two per lane).
constexpr int kWave2GivensMax = 127;

// givens_wave for kWaveGivensMax < k <= kWave2GivensMax: every per-lane quantity is held
// as two entries (lane and lane + 64). Same arithmetic, in the same order, as
// givens_step.
template <int NE>
__device__ inline void givens_wave_n(double *H, int ld, double *R, double *cs, double *sn,
                                     double *g, double *y, double *rho, double beta, int k,
                                     DevState *st)
{
    const int lane = threadIdx.x & 63;
    const int j = k - 1;
    const double *Hc = H + (size_t)j * ld;
    double *Rc = R + (size_t)j * ld;
    const bool bd = st->bd_k == k;
    double hv[NE], cv[NE], sv[NE], gl[NE], rv[NE], yv[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const int r = e * 64 + lane;
        hv[e] = r <= k ? ((r == k && bd) ? 0.0 : Hc[r]) : 0.0;
        cv[e] = r < j ? cs[r] : 0.0;
        sv[e] = r < j ? sn[r] : 0.0;
        gl[e] = r < k ? g[r] : 0.0;
        rv[e] = 0.0;
        yv[e] = 0.0;
    }
    // rotations 0..j-1 applied to the column: t carries entry i+1 down the column
    double t = readlane_n(hv, 0);
    for (int i = 0; i < j; ++i) {
        const double a = t, b = readlane_n(hv, i + 1);
        const double ci = readlane_n(cv, i), si = readlane_n(sv, i);
        const double o = ci * a + si * b;
        t = -si * a + ci * b;
#pragma unroll
        for (int e = 0; e < NE; ++e)
            if (e * 64 + lane == i) rv[e] = o;
    }
    const double a = t, b = readlane_n(hv, k);
    const double r = hypot(a, b);
    double c = 1.0, s = 0.0;
    if (r > 0.0) {
        c = a / r;
        s = b / r;
    } else if (lane == 0) {
        st->error |= 4;
    }
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const int ri = e * 64 + lane;
        if (ri == j) rv[e] = r;
        if (ri < k) Rc[ri] = rv[e];
        if (ri == k) Rc[k] = 0.0;
    }
    const double gj = readlane_n(gl, j);
    if (lane == 0) {
        cs[j] = c;
        sn[j] = s;
        g[j] = c * gj;
        g[k] = -s * gj;
        st->ls = fabs(-s * gj);
        st->k = k;
    }
#pragma unroll
    for (int e = 0; e < NE; ++e)
        if (e * 64 + lane == j) gl[e] = c * gj;
    // back substitution R_k y = g[0..k), column by column from the last
    for (int jb = j; jb >= 0; jb -= 8) {
        double col[8][NE];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int jj = jb - u;
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const int ri = e * 64 + lane;
                col[u][e] = jj < 0 ? 0.0
                                   : (jj == j ? rv[e]
                                              : (ri <= jj ? R[(size_t)jj * ld + ri] : 0.0));
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int jj = jb - u;
            if (jj < 0) break;
            const double yj = readlane_n(gl, jj) / readlane_n(col[u], jj);
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const int ri = e * 64 + lane;
                if (ri == jj) yv[e] = yj;
                if (ri < jj) gl[e] -= col[u][e] * yj;
            }
        }
    }
#pragma unroll
    for (int e = 0; e < NE; ++e)
        if (e * 64 + lane < k) y[e * 64 + lane] = yv[e];
    if (rho) {
        double acc[NE];
#pragma unroll
        for (int e = 0; e < NE; ++e) acc[e] = e * 64 + lane == 0 ? beta : 0.0;
        for (int jj = 0; jj < k; ++jj) {
            const double yj = readlane_n(yv, jj);
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const int ri = e * 64 + lane;
                if (ri <= k && jj >= ri - 1) acc[e] -= H[(size_t)jj * ld + ri] * yj;
            }
        }
#pragma unroll
        for (int e = 0; e < NE; ++e)
            if (e * 64 + lane <= k) rho[e * 64 + lane] = acc[e];
    }
}

// After the normalisation, by the block of rank 0 of a single solve's launch: step 0
// sets beta = ||r_0|| (or raises the zero-right-hand-side stop), step k >= 1 runs the
// Givens update of column k, then copies the scalars to the host slot.
__device__ inline void mgs_tail(const MgsDev &a, int rank)
{
    if (rank != 0) return;
    DevState *st = a.st;
    if (a.set_beta && threadIdx.x == 0 && !st->error) {
        if (st->hnext == 0.0) {
            st->stop = 1;
            st->stop_k = 0;
            st->stop_reason = kStopZero;
        } else {
            st->beta = st->hnext;
        }
    }
    if (a.giv.H) {
        __syncthreads();   // h_{1..k+1,k} and the breakdown flag, written by thread 0
        const GivensDev &g = a.giv;
        if (a.step <= kWaveGivensMax) {
            if (threadIdx.x < 64)
                givens_wave(g.H, g.ld, g.R, g.cs, g.sn, g.g, g.y, g.rho, st->beta, a.step, st);
        } else if (a.step <= kWave2GivensMax) {
            if (threadIdx.x < 64)
                givens_wave_n<2>(g.H, g.ld, g.R, g.cs, g.sn, g.g, g.y, g.rho, st->beta, a.step,
                                 st);
        } else {
            givens_step<kBlock>(g.H, g.ld, g.R, g.cs, g.sn, g.g, g.y, g.rho, st->beta, a.step,
                                st);
            __syncthreads();
        }
        if (g.snap && threadIdx.x == 0) *g.snap = *st;
    }
}

// Rank r owns the E*kBlock consecutive elements from r*E*kBlock; register e of a lane
// holds element base + e*kBlock, so every register is a coalesced wave access at a
// compile-time offset from one per-lane address. The G ranks cover G*E*kBlock >= L
// elements: the buffers are allocated that long and q is zero past L (the padding is
// cleared once per solve), so there are no bounds tests and the padding of w_{k+1}
// comes out zero.
// Low-synchronisation sweep of step k (2 <= k <= kIcwyMaxK) for mgs_body: leaves q_k
// minus its projections in qv, sets qq = ||q_k||^2, writes h_{1..k,k} and the new Gram row
// (rank 0). Same element ownership as mgs_body.
template <typename TX, typename TV, int E>
__device__ inline void mgs_icwy_sweep(const MgsDev &a, int rank, int G, double (&qv)[E],
                                      double *tab, IcwyLds &il, double *lds, double &qq)
{
    const int k = a.k;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const size_t base = (size_t)rank * (E * kBlock) + threadIdx.x;
    const TV *V = static_cast<const TV *>(a.V) + base;
    const TV *wk = V + (size_t)(k - 1) * a.ldv;
    int *err = &a.st->error;
    // Gram rows 0..k-2 (earlier steps) into LDS while the sweep runs
    const int ntri = (k - 1) * (k - 2) / 2;
    {
        // all loads issued at once (clamped into the rows written so far)
        constexpr int kTriPer = (kIcwyMaxK * (kIcwyMaxK - 1) / 2 + kBlock - 1) / kBlock;
        double tv[kTriPer];
#pragma unroll
        for (int u = 0; u < kTriPer; ++u)
            tv[u] = a.gram[min((int)threadIdx.x + u * kBlock, max(ntri - 1, 0))];
#pragma unroll
        for (int u = 0; u < kTriPer; ++u)
            if ((int)threadIdx.x + u * kBlock < ntri) il.tri[threadIdx.x + u * kBlock] = tv[u];
    }
    constexpr bool kHold = E < 32;
    TV wkv[kHold ? E : 1];
    if constexpr (kHold) {
#pragma unroll
        for (int e = 0; e < E; ++e) wkv[e] = wk[e * kBlock];
    }
    double s2 = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) s2 = fma(qv[e], qv[e], s2);
    // D basis vectors per trip, all their loads issued before any is used (a trip then
    // costs one memory latency); past the last vector the loads repeat it, unused
    constexpr int D = E >= 32 ? 1 : (32 / E < 8 ? 32 / E : 8);
    for (int i0 = 0; i0 < k; i0 += D) {
        TV wb[D][E];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const TV *w = V + (size_t)min(i0 + d, k - 1) * a.ldv;
#pragma unroll
            for (int e = 0; e < E; ++e) wb[d][e] = w[e * kBlock];
        }
        // the trip's 2D wave sums form one straight-line block, so that their lane
        // exchanges overlap; sums past the last vector are computed and dropped
        double ds[D], dl[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            ds[d] = 0.0;
            dl[d] = 0.0;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const double we = to_f64(wb[d][e]);
                ds[d] = fma(qv[e], we, ds[d]);
                if constexpr (kHold) dl[d] = fma(to_f64(wkv[e]), we, dl[d]);
                else dl[d] = fma(to_f64(wk[e * kBlock]), we, dl[d]);
            }
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            ds[d] = wave_sum_dpp(ds[d]);
            dl[d] = wave_sum_dpp(dl[d]);
        }
        if (lane == 0) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const int i = i0 + d;
                if (i < k) il.part[wave][i] = ds[d];
                if (i < k - 1) il.part[wave][k + 1 + i] = dl[d];
            }
        }
    }
    s2 = wave_sum_dpp(s2);
    if (lane == 0) il.part[wave][k] = s2;
    __syncthreads();
    const int R = 2 * k;
    double mine = 0.0;
    if ((int)threadIdx.x < R) {
        mine = il.part[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) mine += il.part[w][threadIdx.x];
    }
    if (G == 1) {
        if ((int)threadIdx.x < R) il.tot[threadIdx.x] = mine;
        __syncthreads();
    } else {
        if ((int)threadIdx.x < R) publish(tab + (size_t)threadIdx.x * G + rank, mine);
        gather_rows(tab, G, R, il.red, il.tot, lds, err);
    }
    qq = il.tot[k];
    // forward substitution by the first wave, column by column: lane j holds h_j and
    // subtracts <w_j, w_i> h_i once h_i is final (h_i broadcast by readlane); the same
    // arithmetic, in the same order, in every block
    if (wave == 0) {
        double hj = lane < k ? il.tot[lane] : 0.0;
        const double *lrow = lane < k - 1 ? il.tri + lane * (lane - 1) / 2 : il.tot + k + 1;
        for (int i = 0; i < k - 1; ++i) {
            const double hi = readlane_d(hj, i);
            if (lane > i && lane < k) hj = fma(-lrow[i], hi, hj);
        }
        if (lane < k) il.h[lane] = hj;
    }
    __syncthreads();
    if (rank == 0) {
        if ((int)threadIdx.x < k) a.hcol[threadIdx.x] = il.h[threadIdx.x];
        if ((int)threadIdx.x < k - 1) a.gram[ntri + threadIdx.x] = il.tot[k + 1 + threadIdx.x];
    }
    for (int i0 = 0; i0 < k; i0 += D) {
        TV wb[D][E];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const TV *w = V + (size_t)min(i0 + d, k - 1) * a.ldv;
#pragma unroll
            for (int e = 0; e < E; ++e) wb[d][e] = w[e * kBlock];
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (i0 + d >= k) break;
            const double h = il.h[i0 + d];
#pragma unroll
            for (int e = 0; e < E; ++e) qv[e] = fma(-h, to_f64(wb[d][e]), qv[e]);
        }
    }
}

template <typename TX, typename TV, int E>
__device__ inline void mgs_body(const MgsDev &a, int rank, int G, double *lds,
                                IcwyLds *il = nullptr)
{
    const size_t base = (size_t)rank * (E * kBlock) + threadIdx.x;
    const TX *q = static_cast<const TX *>(a.q) + base;
    int *err = &a.st->error;
    // Large tiles read w_i again after the reduction (an L2 hit) instead of holding it
    // across the barrier, which halves their register footprint.
    constexpr bool kReload = E >= 32;
    constexpr int EW = kReload ? 1 : E;
    double qv[E];
    TV wv[EW];
#pragma unroll
    for (int e = 0; e < E; ++e) qv[e] = to_f64(q[e * kBlock]);
    double *tab = a.partials + (size_t)(a.step & 1) * a.rows * G;
    double *next = a.partials + (size_t)((a.step + 1) & 1) * a.rows * G;
    // rows the next step uses: up to 2(k+1) in the low-synchronisation form
    const bool icwy = a.gram && il && a.k >= 2 && a.k <= kIcwyMaxK;
    const int clear_to = a.gram ? 2 * a.k + 2 : a.k + 2;
    if (threadIdx.x == 0) {
        const double empty = __longlong_as_double((long long)kSlotEmpty);
        for (int r = 0; r <= clear_to && r < a.rows; ++r)
            __hip_atomic_store(next + (size_t)r * G + rank, empty, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    // a group of one block: its block sums are the totals, no exchange through memory
    const bool solo = G == 1;
    double qq = 0.0, h = 0.0;
    const int norm_row = icwy ? 2 * a.k : a.k;
    if (icwy) {
        mgs_icwy_sweep<TX, TV, E>(a, rank, G, qv, tab, *il, lds, qq);
    } else {
    // small tiles: w_{i+1} is loaded while the partial sums of <q, w_i> are exchanged
    TV wn[EW];
    if constexpr (!kReload) {
        if (a.k > 0) {
#pragma unroll
            for (int e = 0; e < E; ++e) wn[e] = static_cast<const TV *>(a.V)[base + e * kBlock];
        }
    }
    for (int i = 0; i < a.k; ++i) {
        const TV *w = static_cast<const TV *>(a.V) + (size_t)i * a.ldv + base;
        double d = 0.0, s2 = 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            TV we;
            if constexpr (kReload) {
                we = w[e * kBlock];
            } else {
                we = wn[e];
                wv[e] = we;
            }
            d = fma(qv[e], to_f64(we), d);
            if (i == 0) s2 = fma(qv[e], qv[e], s2);
        }
        if constexpr (!kReload) {
            if (i + 1 < a.k) {
#pragma unroll
                for (int e = 0; e < E; ++e) wn[e] = w[a.ldv + e * kBlock];
            }
        }
        d = block_sum(d, lds);
        if (i == 0) s2 = block_sum(s2, lds);
        if (solo) {
            h = d;
            if (i == 0) qq = s2;
        } else {
            if (threadIdx.x == 0) {
                publish(tab + (size_t)i * G + rank, d);
                if (i == 0) publish(tab + (size_t)(a.k + 1) * G + rank, s2);
            }
            h = gather_total(tab + (size_t)i * G, G, lds, err);
            if (i == 0) qq = gather_total(tab + (size_t)(a.k + 1) * G, G, lds, err);
        }
        if (rank == 0 && threadIdx.x == 0) a.hcol[i] = h;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if constexpr (kReload) qv[e] = fma(-h, to_f64(w[e * kBlock]), qv[e]);
            else qv[e] = fma(-h, to_f64(wv[e]), qv[e]);
        }
    }
    }
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) s = fma(qv[e], qv[e], s);
    s = block_sum(s, lds);
    double hn2 = s;
    if (!solo) {
        if (threadIdx.x == 0) publish(tab + (size_t)norm_row * G + rank, s);
        hn2 = gather_total(tab + (size_t)norm_row * G, G, lds, err);
    }
    if (a.k == 0) qq = hn2;
    const double hn = sqrt(hn2);
    const double q0 = sqrt(qq);
    const bool finite = isfinite(hn) && isfinite(q0);
    const bool bd = !(hn > a.bd_rel * q0);
    if (rank == 0 && threadIdx.x == 0) {
        a.hcol[a.k] = hn;
        a.st->hnext = hn;
        a.st->qnorm0 = q0;
        if (bd && a.step > 0) a.st->bd_k = a.step;
        if (!finite) a.st->error |= 2;
    }
    TV *vo = static_cast<TV *>(a.vout) + base;
    TX *cu = static_cast<TX *>(a.cur) + base;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const TV w = (bd || !finite) ? zero_of<TV>() : from_f64<TV>(qv[e] / hn);
        vo[e * kBlock] = w;
        cu[e * kBlock] = (TX)to_f64(w);
    }
}


// The same orthogonalisation for vectors too long to keep in the registers of one
// resident block group: q_k lives in an FP64 scratch vector (a.q64, zero-padded like the
// other vectors) and every stage is one pass over it. Pass i updates q -= h_{i-1} w_{i-1}
// and accumulates <q, w_i> (or ||q||^2 after the last basis vector), so a stage reads q,
// w_{i-1} and w_i and writes q once. Block `rank` takes elements rank*kBlock + t +
// j*G*kBlock; reductions are the same fixed-order group reductions as above.
template <typename TX, typename TV>
__device__ inline void mgs_stream_body(const MgsDev &a, int rank, int G, double *lds)
{
    double *q64 = a.q64;
    const size_t T = (size_t)G * kBlock;
    const size_t L = (size_t)a.L;
    const TX *q = static_cast<const TX *>(a.q);
    const TV *V = static_cast<const TV *>(a.V);
    int *err = &a.st->error;
    double *tab = a.partials + (size_t)(a.step & 1) * a.rows * G;
    double *next = a.partials + (size_t)((a.step + 1) & 1) * a.rows * G;
    if (threadIdx.x == 0) {
        const double empty = __longlong_as_double((long long)kSlotEmpty);
        for (int r = 0; r <= a.k + 2 && r < a.rows; ++r)
            __hip_atomic_store(next + (size_t)r * G + rank, empty, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    // pass 0: q64 = q, <q, w_1> and ||q||^2 (or only ||q||^2 when k = 0); every pass
    // keeps kSU elements per thread in flight
    constexpr int kSU = 4;
    double d = 0.0, s2 = 0.0;
    const TV *w0 = V;
    for (size_t l0 = (size_t)rank * kBlock + threadIdx.x; l0 < L; l0 += kSU * T) {
        double v[kSU], w[kSU];
#pragma unroll
        for (int u = 0; u < kSU; ++u) {
            const size_t l = l0 + u * T;
            v[u] = l < L ? to_f64(q[l]) : 0.0;
            w[u] = (l < L && a.k > 0) ? to_f64(w0[l]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kSU; ++u) {
            const size_t l = l0 + u * T;
            if (l < L) q64[l] = v[u];
            s2 = fma(v[u], v[u], s2);
            d = fma(v[u], w[u], d);
        }
    }
    double qq;
    double hprev = 0.0;
    if (a.k > 0) {
        d = block_sum(d, lds);
        s2 = block_sum(s2, lds);
        if (threadIdx.x == 0) {
            publish(tab + rank, d);
            publish(tab + (size_t)(a.k + 1) * G + rank, s2);
        }
        hprev = gather_total(tab, G, lds, err);
        qq = gather_total(tab + (size_t)(a.k + 1) * G, G, lds, err);
        if (rank == 0 && threadIdx.x == 0) a.hcol[0] = hprev;
    } else {
        s2 = block_sum(s2, lds);
        if (threadIdx.x == 0) publish(tab + rank, s2);
        qq = gather_total(tab, G, lds, err);
    }
    double hn2 = qq;
    for (int i = 1; i <= a.k; ++i) {
        // q -= h_{i-1} w_{i-1}, then <q, w_i> (i < k) or ||q||^2 (i = k)
        const TV *wp = V + (size_t)(i - 1) * a.ldv;
        const TV *wi = V + (size_t)i * a.ldv;
        const bool last = i == a.k;
        double acc = 0.0;
        for (size_t l0 = (size_t)rank * kBlock + threadIdx.x; l0 < L; l0 += kSU * T) {
            double v[kSU], w[kSU];
#pragma unroll
            for (int u = 0; u < kSU; ++u) {
                const size_t l = l0 + u * T;
                const bool in = l < L;
                v[u] = in ? fma(-hprev, to_f64(wp[l]), q64[l]) : 0.0;
                w[u] = (in && !last) ? to_f64(wi[l]) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kSU; ++u) {
                const size_t l = l0 + u * T;
                if (l < L) q64[l] = v[u];
                acc = last ? fma(v[u], v[u], acc) : fma(v[u], w[u], acc);
            }
        }
        acc = block_sum(acc, lds);
        if (threadIdx.x == 0) publish(tab + (size_t)i * G + rank, acc);
        const double h = gather_total(tab + (size_t)i * G, G, lds, err);
        if (last) {
            hn2 = h;
        } else {
            hprev = h;
            if (rank == 0 && threadIdx.x == 0) a.hcol[i] = h;
        }
    }
    const double hn = sqrt(hn2);
    const double q0 = sqrt(qq);
    const bool finite = isfinite(hn) && isfinite(q0);
    const bool bd = !(hn > a.bd_rel * q0);
    if (rank == 0 && threadIdx.x == 0) {
        a.hcol[a.k] = hn;
        a.st->hnext = hn;
        a.st->qnorm0 = q0;
        if (bd && a.step > 0) a.st->bd_k = a.step;
        if (!finite) a.st->error |= 2;
    }
    TV *vo = static_cast<TV *>(a.vout);
    TX *cu = static_cast<TX *>(a.cur);
    for (size_t l0 = (size_t)rank * kBlock + threadIdx.x; l0 < L; l0 += kSU * T) {
        double v[kSU];
#pragma unroll
        for (int u = 0; u < kSU; ++u) {
            const size_t l = l0 + u * T;
            v[u] = l < L ? q64[l] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kSU; ++u) {
            const size_t l = l0 + u * T;
            if (l < L) {
                const TV w = (bd || !finite) ? zero_of<TV>() : from_f64<TV>(v[u] / hn);
                vo[l] = w;
                cu[l] = (TX)to_f64(w);
            }
        }
    }
}


}  // namespace
}  // namespace abg
