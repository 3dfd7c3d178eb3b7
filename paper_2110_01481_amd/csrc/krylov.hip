// Arnoldi machinery of AB-/BA-GMRES (Sec. 2) for gfx950:
//   mgs     modified Gram-Schmidt of q_k against w_1..w_k, h_{k+1,k} = ||q_k||,
//           w_{k+1} = q_k / h_{k+1,k}; one launch per Arnoldi step whose blocks all stay
//           resident, keep q_k in FP64 registers, read each basis vector once, and take
//           one group-wide reduction per inner product (the sequential loop over i of
//           modified Gram-Schmidt is kept).
//   givens  FP64 Givens update of the Hessenberg least squares problem, back
//           substitution for y_k and the small residual vector ||r_0|| e_1 - H_k y_k.
//   combine basis combinations base + sum_j c_j v_j (iterates and residual vectors)
//           with FP64 accumulation and a fixed-order norm reduction.
// Every reduction runs in a fixed order, so results are identical run to run.
#include <cmath>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <unordered_map>

#include <hip/hip_ext.h>

#include "krylov_body.h"

namespace abg {
namespace {

constexpr int kCombU = 4;
constexpr int kCombJ = 4;   // basis columns per trip of the combination

// Ranks are handed out in the order blocks start, so the blocks holding ranks are
// running; a group no larger than the blocks the device holds at once always completes
// (an ordinary launch then needs no co-scheduling guarantee).
template <typename TX, typename TV, int E>
__global__ __launch_bounds__(kBlock) void mgs_kernel(MgsDev a)
{
    __shared__ double lds[kWaves];
    __shared__ IcwyLds il;
    __shared__ int s_rank;
    if (halted(a.st, a.step)) {
        if (a.giv.snap && blockIdx.x == 0 && threadIdx.x == 0) *a.giv.snap = *a.st;
        return;
    }
    if (threadIdx.x == 0)
        s_rank = (int)__hip_atomic_fetch_add(a.ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int rank = __builtin_amdgcn_readfirstlane(s_rank);
    mgs_body<TX, TV, E>(a, rank, gridDim.x, lds, &il);
    mgs_tail(a, rank);
}

template <typename TX, typename TV>
__global__ __launch_bounds__(kBlock) void mgs_stream_kernel(MgsDev a)
{
    __shared__ double lds[kWaves];
    __shared__ int s_rank;
    if (halted(a.st, a.step)) {
        if (a.giv.snap && blockIdx.x == 0 && threadIdx.x == 0) *a.giv.snap = *a.st;
        return;
    }
    if (threadIdx.x == 0)
        s_rank = (int)__hip_atomic_fetch_add(a.ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int rank = __builtin_amdgcn_readfirstlane(s_rank);
    mgs_stream_body<TX, TV>(a, rank, gridDim.x, lds);
    mgs_tail(a, rank);
}

// ---- resident-block bookkeeping -----------------------------------------------------
struct CapInfo {
    int max_blocks = 0;
};
std::mutex g_cap_mu;
std::unordered_map<const void *, CapInfo> g_cap;

hipError_t resident_capacity(const void *fn, int *max_blocks)
{
    std::lock_guard<std::mutex> lk(g_cap_mu);
    auto it = g_cap.find(fn);
    if (it != g_cap.end()) {
        *max_blocks = it->second.max_blocks;
        return hipSuccess;
    }
    int dev = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, 0);
    if (e != hipSuccess) return e;
    CapInfo ci;
    ci.max_blocks = per_cu * prop.multiProcessorCount;
    g_cap[fn] = ci;
    *max_blocks = ci.max_blocks;
    return hipSuccess;
}

// Blocks of the MGS launch when the vector is long enough (fewer blocks make
// the grid-wide reductions cheaper, more blocks keep more loads in flight). The
// environment variable ABG_MGS_BLOCKS overrides it.
int default_target_blocks()
{
    const char *e = getenv("ABG_MGS_BLOCKS");
    const int v = e ? atoi(e) : 0;
    return v > 0 ? v : 256;
}
int g_target_blocks = default_target_blocks();
int g_force_stream = 0;

// Streaming variant: a group of at most kStreamBlocks resident blocks.
constexpr int kStreamBlocks = 512;

// e0, e1: events stamped with the kernel's start and end (timing), or null
template <typename TX, typename TV>
hipError_t mgs_stream_go(const MgsDev &d, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (!d.q64) return hipErrorInvalidValue;
    const void *fn = reinterpret_cast<const void *>(&mgs_stream_kernel<TX, TV>);
    int cap = 0;
    hipError_t e = resident_capacity(fn, &cap);
    if (e != hipSuccess) return e;
    const int G = std::min(kStreamBlocks, cap);
    hipExtLaunchKernelGGL(mgs_stream_kernel<TX, TV>, dim3(G), dim3(kBlock), 0, s, e0, e1, 0, d);
    return hipGetLastError();
}

template <typename TX, typename TV, int E>
hipError_t mgs_go(const MgsDev &d, int G, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    const void *fn = reinterpret_cast<const void *>(&mgs_kernel<TX, TV, E>);
    int cap = 0;
    hipError_t e = resident_capacity(fn, &cap);
    if (e != hipSuccess) return e;
    if (G > cap || G > kMaxGrid || (g_force_stream && d.q64)) {
        // q_k does not fit the registers of the blocks the device holds at once
        if (d.q64) return mgs_stream_go<TX, TV>(d, s, e0, e1);
        return hipErrorCooperativeLaunchTooLarge;
    }
    hipExtLaunchKernelGGL(mgs_kernel<TX, TV, E>, dim3(G), dim3(kBlock), 0, s, e0, e1, 0, d);
    return hipGetLastError();
}

template <typename TX, typename TV>
hipError_t mgs_dispatch(const MgsDev &d, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    // A vector one block can hold in its registers gets one block: its reductions stay
    // inside the CU, where a reduction across the XCDs costs several microseconds. Longer
    // vectors: the smallest register tile E per thread such that target blocks cover L;
    // beyond the largest tile the grid grows instead.
    const long long L = d.L;
    const int maxE = sizeof(TV) == 8 ? 32 : 64;
    int E = 1;
    if (L <= (long long)kBlock * maxE) {
        while ((long long)kBlock * E < L) E *= 2;
    } else {
        while (E < maxE && (long long)g_target_blocks * kBlock * E < L) E *= 2;
    }
    long long G = (L + (long long)kBlock * E - 1) / ((long long)kBlock * E);
    if (G < 1) G = 1;
    const int Gi = (int)G;
    switch (E) {
    case 1: return mgs_go<TX, TV, 1>(d, Gi, s, e0, e1);
    case 2: return mgs_go<TX, TV, 2>(d, Gi, s, e0, e1);
    case 4: return mgs_go<TX, TV, 4>(d, Gi, s, e0, e1);
    case 8: return mgs_go<TX, TV, 8>(d, Gi, s, e0, e1);
    case 16: return mgs_go<TX, TV, 16>(d, Gi, s, e0, e1);
    case 32: return mgs_go<TX, TV, 32>(d, Gi, s, e0, e1);
    default:
        if constexpr (sizeof(TV) < 8) return mgs_go<TX, TV, 64>(d, Gi, s, e0, e1);
        return hipErrorInvalidValue;
    }
}

// ---- combinations, norms -------------------------------------------------------------
template <typename TO, typename TB, typename TV>
__global__ __launch_bounds__(kBlock) void combine_kernel(const TB *__restrict__ base, double bcoef,
                                                         const TV *__restrict__ V, size_t ldv,
                                                         int kk, const double *__restrict__ coef,
                                                         double sgn, TO *__restrict__ out,
                                                         long long L, double *partials,
                                                         unsigned *count, double *norm,
                                                         DevState *st, int k, DevState *snap)
{
    __shared__ double cf[kMaxCoef];
    __shared__ double lds[kWaves];
    __shared__ int last;
    if (halted(st, k)) {
        if (snap && blockIdx.x == 0 && threadIdx.x == 0) *snap = *st;
        return;
    }
    for (int j = threadIdx.x; j < kk; j += kBlock) cf[j] = sgn * coef[j];
    __syncthreads();
    // each thread combines kCombU elements per trip, all of a column's loads in flight
    const long long T = (long long)gridDim.x * kBlock;
    double ss = 0.0;
    for (long long l0 = (long long)blockIdx.x * kBlock + threadIdx.x; l0 < L; l0 += kCombU * T) {
        double acc[kCombU];
        bool in[kCombU];
#pragma unroll
        for (int u = 0; u < kCombU; ++u) {
            const long long l = l0 + u * T;
            in[u] = l < L;
            acc[u] = (in[u] && base) ? bcoef * to_f64(base[l]) : 0.0;
        }
        // four columns' loads in flight at once; each element still sums over j in order
        int j = 0;
        for (; j + kCombJ <= kk; j += kCombJ) {
            double x[kCombJ][kCombU];
#pragma unroll
            for (int jj = 0; jj < kCombJ; ++jj) {
                const TV *v = V + (size_t)(j + jj) * ldv + l0;
#pragma unroll
                for (int u = 0; u < kCombU; ++u) x[jj][u] = in[u] ? to_f64(v[u * T]) : 0.0;
            }
#pragma unroll
            for (int jj = 0; jj < kCombJ; ++jj) {
#pragma unroll
                for (int u = 0; u < kCombU; ++u) acc[u] = fma(cf[j + jj], x[jj][u], acc[u]);
            }
        }
        for (; j < kk; ++j) {
            const TV *v = V + (size_t)j * ldv + l0;
            double x[kCombU];
#pragma unroll
            for (int u = 0; u < kCombU; ++u) x[u] = in[u] ? to_f64(v[u * T]) : 0.0;
#pragma unroll
            for (int u = 0; u < kCombU; ++u) acc[u] = fma(cf[j], x[u], acc[u]);
        }
#pragma unroll
        for (int u = 0; u < kCombU; ++u) {
            if (in[u]) {
                out[l0 + u * T] = (TO)acc[u];
                ss = fma(acc[u], acc[u], ss);
            }
        }
    }
    if (!norm) return;
    // fixed-order norm: per-block partials, summed by the last block to finish
    ss = block_sum(ss, lds);
    if (threadIdx.x == 0) {
        agent_store(partials + blockIdx.x, ss);
        const unsigned prev = __hip_atomic_fetch_add(count, 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        last = prev == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    last_block_fence();
    double t = 0.0;
    for (int j = threadIdx.x; j < (int)gridDim.x; j += kBlock) t += agent_load(partials + j);
    t = block_sum(t, lds);
    if (threadIdx.x == 0) {
        __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const double r = sqrt(t);
        *norm = r;
        if (st) {
            if (!isfinite(r)) {
                st->error |= 2;
            } else if (st->dp_thr > 0.0 && r <= st->dp_thr && !st->stop) {
                st->stop = 1;
                st->stop_k = k;
                st->stop_reason = kStopDP;
            }
            if (snap) *snap = *st;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void sub_norm_kernel(const T *__restrict__ a, const T *__restrict__ b,
                                                          T *__restrict__ out, long long L,
                                                          double *partials)
{
    __shared__ double lds[kWaves];
    const long long T_ = (long long)gridDim.x * kBlock;
    double ss = 0.0;
    for (long long l = (long long)blockIdx.x * kBlock + threadIdx.x; l < L; l += T_) {
        const double v = (double)a[l] - (double)b[l];
        out[l] = (T)v;
        ss = fma(v, v, ss);
    }
    ss = block_sum(ss, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = ss;
}

__global__ __launch_bounds__(kBlock) void reduce_sqrt_kernel(const double *partials, int nb, double *dst)
{
    __shared__ double lds[kWaves];
    double s = 0.0;
    for (int j = threadIdx.x; j < nb; j += kBlock) s += partials[j];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) *dst = sqrt(s);
}

template <typename T>
__global__ void axpy_inplace_kernel(T *x, const T *x0, long long L)
{
    const long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (l < L) x[l] = (T)((double)x[l] + (double)x0[l]);
}

__global__ void fill_u32_kernel(unsigned *p, size_t n, unsigned v)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void fill_f64_kernel(double *p, size_t n, double v)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// The ranges of a fused initialisation, one after the other over the whole grid, and the
// initial scalars (written by one thread).
struct FillList {
    FillRange r[kMaxFill];
    int n;
    int has_init;
    DevState init;
};

__global__ __launch_bounds__(kBlock) void init_fill_kernel(const FillList L, DevState *st)
{
    const size_t T = (size_t)gridDim.x * kBlock;
    const size_t i0 = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (L.has_init && i0 == 0) *st = L.init;
    for (int r = 0; r < L.n; ++r) {
        unsigned *p = static_cast<unsigned *>(L.r[r].p);
        const unsigned *src = static_cast<const unsigned *>(L.r[r].src);
        const size_t n = L.r[r].n, ns = L.r[r].n_src;
        const unsigned lo = L.r[r].lo, hi = L.r[r].hi;
        for (size_t i = i0; i < n; i += T) p[i] = i < ns ? src[i] : ((i & 1) ? hi : lo);
    }
}

__global__ __launch_bounds__(64) void givens_kernel(double *H, int ld, double *R, double *cs,
                                                    double *sn, double *g, double *y,
                                                    double *rho, const double *beta, int k,
                                                    DevState *st, DevState *snap)
{
    if (halted(st, k)) {
        if (snap && threadIdx.x == 0) *snap = *st;
        return;
    }
    if (k <= kWaveGivensMax) {
        givens_wave(H, ld, R, cs, sn, g, y, rho, *beta, k, st);
    } else {
        givens_step(H, ld, R, cs, sn, g, y, rho, *beta, k, st);
        __syncthreads();
    }
    if (snap && threadIdx.x == 0) *snap = *st;
}

// After the initial normalisation: beta = ||r_0|| for the later steps, or (r_0 = 0) the
// zero-right-hand-side stop before step 1.
__global__ void set_beta_kernel(DevState *st)
{
    if (threadIdx.x != 0 || st->error) return;
    if (st->hnext == 0.0) {
        st->stop = 1;
        st->stop_k = 0;
        st->stop_reason = kStopZero;
    } else {
        st->beta = st->hnext;
    }
}

__global__ void clear_stop_kernel(DevState *st)
{
    if (threadIdx.x == 0) {
        st->stop = 0;
        st->stop_k = 0;
        st->stop_reason = kStopNone;
    }
}

int blocks_for(long long L, long long cap = 1024)
{
    long long b = (L + kBlock - 1) / kBlock;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (int)b;
}

template <typename TO, typename TB, typename TV>
hipError_t combine_go(const void *base, double bcoef, const void *V, size_t ldv, int kk,
                      const double *coef, double sgn, void *out, long long L, double *partials,
                      unsigned *count, double *norm, DevState *st, int k, DevState *snap,
                      hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    // with a norm, every block signals completion on one counter: keep the grid moderate
    const int nb = blocks_for((L + kCombU - 1) / kCombU, norm ? 512 : 1024);
    hipExtLaunchKernelGGL(combine_kernel<TO, TB, TV>, dim3(nb), dim3(kBlock), 0, s, e0, e1, 0,
                          static_cast<const TB *>(base), bcoef, static_cast<const TV *>(V), ldv,
                          kk, coef, sgn, static_cast<TO *>(out), L, partials, count, norm, st, k,
                          snap);
    return hipGetLastError();
}

// Share of the device (GroupBudget units) of the Gram-Schmidt launch mgs_dispatch makes
// for vectors of length L: the same tile and group choice, then the group's blocks
// against what the device holds of that kernel.
template <typename TX, typename TV>
hipError_t group_units_t(long long L, bool q64, long long *units)
{
    const int maxE = sizeof(TV) == 8 ? 32 : 64;
    int E = 1;
    if (L <= (long long)kBlock * maxE) {
        while ((long long)kBlock * E < L) E *= 2;
    } else {
        while (E < maxE && (long long)g_target_blocks * kBlock * E < L) E *= 2;
    }
    long long G = (L + (long long)kBlock * E - 1) / ((long long)kBlock * E);
    *units = 0;
    if (G <= 1) return hipSuccess;
    const void *fn = nullptr;
    switch (E) {
    case 1: fn = reinterpret_cast<const void *>(&mgs_kernel<TX, TV, 1>); break;
    case 2: fn = reinterpret_cast<const void *>(&mgs_kernel<TX, TV, 2>); break;
    case 4: fn = reinterpret_cast<const void *>(&mgs_kernel<TX, TV, 4>); break;
    case 8: fn = reinterpret_cast<const void *>(&mgs_kernel<TX, TV, 8>); break;
    case 16: fn = reinterpret_cast<const void *>(&mgs_kernel<TX, TV, 16>); break;
    case 32: fn = reinterpret_cast<const void *>(&mgs_kernel<TX, TV, 32>); break;
    default:
        if constexpr (sizeof(TV) < 8) fn = reinterpret_cast<const void *>(&mgs_kernel<TX, TV, 64>);
        break;
    }
    if (!fn) return hipErrorInvalidValue;
    int cap = 0;
    hipError_t e = resident_capacity(fn, &cap);
    if (e != hipSuccess) return e;
    if (G > cap || G > kMaxGrid || (g_force_stream && q64)) {
        if (!q64) {
            *units = GroupBudget::kUnits;
            return hipSuccess;
        }
        int caps = 0;
        e = resident_capacity(reinterpret_cast<const void *>(&mgs_stream_kernel<TX, TV>), &caps);
        if (e != hipSuccess) return e;
        *units = GroupBudget::units_for(std::min(kStreamBlocks, caps), caps);
        return hipSuccess;
    }
    *units = GroupBudget::units_for(G, cap);
    return hipSuccess;
}

}  // namespace

void set_mgs_force_stream(int on) { g_force_stream = on ? 1 : 0; }

hipError_t mgs_group_units(int tx, int tv, long long L, bool q64, long long *units)
{
    if (tx == ABG_F64) {
        if (tv == ABG_F64) return group_units_t<double, double>(L, q64, units);
        if (tv == ABG_F32) return group_units_t<double, float>(L, q64, units);
        return group_units_t<double, bf16>(L, q64, units);
    }
    if (tv == ABG_F32) return group_units_t<float, float>(L, q64, units);
    if (tv == ABG_BF16) return group_units_t<float, bf16>(L, q64, units);
    return hipErrorInvalidValue;
}

GroupBudget &device_group_budget()
{
    static std::mutex mu;
    static std::map<int, std::unique_ptr<GroupBudget>> budgets;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    auto &b = budgets[dev];
    if (!b) b.reset(new GroupBudget);
    return *b;
}

void set_mgs_target_blocks(int blocks)
{
    g_target_blocks = blocks < 1 ? 1 : (blocks > kMaxGrid ? kMaxGrid : blocks);
}

hipError_t launch_mgs(const MgsLaunch &m, hipStream_t s)
{
    MgsDev d;
    d.q = m.q;
    d.V = m.V;
    d.ldv = m.ldv;
    d.k = m.k;
    d.L = m.L;
    d.hcol = m.hcol;
    d.vout = m.vout;
    d.cur = m.cur;
    d.partials = m.partials;
    d.rows = m.rows;
    d.ticket = m.ticket;
    d.q64 = m.q64;
    d.st = m.st;
    d.bd_rel = m.bd_rel;
    d.step = m.step;
    d.set_beta = m.set_beta;
    d.gram = m.gram;
    d.giv = GivensDev{m.giv_H, m.giv_R, m.giv_cs, m.giv_sn, m.giv_g, m.giv_y, m.giv_rho,
                      m.giv_ld, m.snap};
    if (m.giv_H && (m.k < 1 || m.k + 1 > kMaxCoef)) return hipErrorInvalidValue;
    // the low-synchronisation form publishes rows 0..2k and clears up to 2k + 2
    if (m.gram && m.rows < 2 * std::min(m.k, kIcwyMaxK) + 3) return hipErrorInvalidValue;
    if (m.snap && !m.giv_H) return hipErrorInvalidValue;
    // timed at the kernel's own start and end when profiling is on
    ProfScope ps(kProfMgs, s, m.step, true);
    if (m.tx == ABG_F64) {
        if (m.tv == ABG_F64) return mgs_dispatch<double, double>(d, s, ps.e0, ps.e1);
        if (m.tv == ABG_F32) return mgs_dispatch<double, float>(d, s, ps.e0, ps.e1);
        return mgs_dispatch<double, bf16>(d, s, ps.e0, ps.e1);
    }
    if (m.tv == ABG_F32) return mgs_dispatch<float, float>(d, s, ps.e0, ps.e1);
    if (m.tv == ABG_BF16) return mgs_dispatch<float, bf16>(d, s, ps.e0, ps.e1);
    return hipErrorInvalidValue;
}

hipError_t launch_combine(int tout, const void *base, double base_coef, int tv, const void *V,
                          size_t ldv, int kk, const double *coef, double sgn, void *out,
                          long long L, double *partials, unsigned *count, double *norm,
                          DevState *st, int k, hipStream_t s, DevState *snap)
{
    if (kk > kMaxCoef) return hipErrorInvalidValue;
    if (snap && !(norm && st)) return hipErrorInvalidValue;
    ProfScope ps(kProfCombine, s, st ? k : 0, true);
#define ABG_COMBINE(TO, TB, TV) \
    combine_go<TO, TB, TV>(base, base_coef, V, ldv, kk, coef, sgn, out, L, partials, count, norm, st, k, \
                           snap, s, ps.e0, ps.e1)
    if (tout == ABG_F64) {
        if (tv == ABG_F64) return ABG_COMBINE(double, double, double);
        if (tv == ABG_F32) return ABG_COMBINE(double, double, float);
        return ABG_COMBINE(double, double, bf16);
    }
    if (tv == ABG_F32) return ABG_COMBINE(float, float, float);
    if (tv == ABG_BF16) return ABG_COMBINE(float, float, bf16);
#undef ABG_COMBINE
    return hipErrorInvalidValue;
}

hipError_t launch_sub_norm(int t, const void *a, const void *b, void *out, long long L,
                           double *partials, int *nblocks, hipStream_t s)
{
    const int nb = blocks_for(L);
    *nblocks = nb;
    if (t == ABG_F64)
        sub_norm_kernel<double><<<nb, kBlock, 0, s>>>(static_cast<const double *>(a), static_cast<const double *>(b),
                                                      static_cast<double *>(out), L, partials);
    else
        sub_norm_kernel<float><<<nb, kBlock, 0, s>>>(static_cast<const float *>(a), static_cast<const float *>(b),
                                                     static_cast<float *>(out), L, partials);
    return hipGetLastError();
}

hipError_t launch_reduce_sqrt(const double *partials, int nb, double *dst, hipStream_t s)
{
    reduce_sqrt_kernel<<<1, kBlock, 0, s>>>(partials, nb, dst);
    return hipGetLastError();
}

hipError_t launch_set_beta(DevState *st, hipStream_t s)
{
    set_beta_kernel<<<1, 64, 0, s>>>(st);
    return hipGetLastError();
}

hipError_t launch_givens(double *H, int ld, double *R, double *cs, double *sn, double *g,
                         double *y, double *rho, const double *beta, int k, DevState *st,
                         hipStream_t s, DevState *snap)
{
    if (k + 1 > kMaxCoef) return hipErrorInvalidValue;
    givens_kernel<<<1, 64, 0, s>>>(H, ld, R, cs, sn, g, y, rho, beta, k, st, snap);
    return hipGetLastError();
}

hipError_t launch_clear_stop(DevState *st, hipStream_t s)
{
    clear_stop_kernel<<<1, 64, 0, s>>>(st);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned *p, size_t n, unsigned v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    fill_u32_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, size_t n, double v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    fill_f64_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_init_fill(const FillRange *r, int n, const DevState *init, DevState *st,
                            hipStream_t s)
{
    if (n < 0 || n > kMaxFill || (init && !st)) return hipErrorInvalidValue;
    FillList L{};
    size_t most = 0;
    for (int i = 0; i < n; ++i) {
        L.r[i] = r[i];
        if (r[i].n_src > r[i].n || (r[i].n && !r[i].p) || (r[i].n_src && !r[i].src))
            return hipErrorInvalidValue;
        most = std::max(most, (size_t)r[i].n);
    }
    L.n = n;
    L.has_init = init != nullptr;
    if (init) L.init = *init;
    const int nb = (int)std::min<size_t>(std::max<size_t>((most + kBlock - 1) / kBlock, 1), 2048);
    init_fill_kernel<<<nb, kBlock, 0, s>>>(L, st);
    return hipGetLastError();
}

unsigned long long slot_empty_bits() { return kSlotEmpty; }

hipError_t launch_clear_slots(double *p, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    double empty;
    const unsigned long long bits = kSlotEmpty;
    memcpy(&empty, &bits, sizeof empty);
    fill_f64_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n, empty);
    return hipGetLastError();
}

hipError_t launch_axpy_inplace(int t, void *x, const void *x0, long long L, hipStream_t s)
{
    const unsigned nb = (unsigned)((L + 255) / 256);
    if (t == ABG_F64)
        axpy_inplace_kernel<double><<<nb, 256, 0, s>>>(static_cast<double *>(x), static_cast<const double *>(x0), L);
    else
        axpy_inplace_kernel<float><<<nb, 256, 0, s>>>(static_cast<float *>(x), static_cast<const float *>(x0), L);
    return hipGetLastError();
}

}  // namespace abg
