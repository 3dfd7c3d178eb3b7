// LSQR (Paige & Saunders) and LSMR (Fong & Saunders): the matched-transpose Krylov
// methods that AB-GMRES and BA-GMRES become when B = A^T (Sec. 5), which the paper runs
// as comparators (Sec. 6.2, Table 6.3). Both rest on Golub-Kahan bidiagonalisation with
// short recurrences (no stored basis):
//     beta_{k+1} u_{k+1} = A v_k - alpha_k u_k,   alpha_{k+1} v_{k+1} = A^T u_{k+1} - beta_{k+1} v_k
// LSQR minimises ||b - A x|| over the Krylov space with one plane rotation per step, LSMR
// minimises ||A^T (b - A x)|| with two. A step is: the forward projection t = A v_k, the
// kernels below, the back projection s = A^T u between them. Scalars are FP64 on the
// device; every block of a vector kernel recomputes a step's rotations from the previous
// values and the last block to finish writes the new ones.
#include "krylov_body.h"

namespace abg {
namespace {

constexpr int kLU = 4;   // elements per thread and trip of the vector kernels

// Reduction of a per-block double to its fixed-order total in the last block to finish
// (true in that block only).
__device__ inline bool last_block_total(double v, double *partials, unsigned *count, double *lds,
                                        double *total, int *last)
{
    v = block_sum(v, lds);
    if (threadIdx.x == 0) {
        agent_store(partials + blockIdx.x, v);
        const unsigned prev = __hip_atomic_fetch_add(count, 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        *last = prev == gridDim.x - 1;
    }
    __syncthreads();
    if (!*last) return false;
    last_block_fence();
    double t = 0.0;
    for (int j = threadIdx.x; j < (int)gridDim.x; j += kBlock) t += agent_load(partials + j);
    t = block_sum(t, lds);
    *total = t;
    if (threadIdx.x == 0) __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

__device__ inline double safe_div(double a, double b) { return b != 0.0 ? a / b : 0.0; }

__device__ inline void dp_check(DevState *st, int k)
{
    if (!isfinite(st->res)) {
        st->error |= 2;
    } else if (st->dp_thr > 0.0 && st->res <= st->dp_thr && !st->stop) {
        st->stop = 1;
        st->stop_k = k;
        st->stop_reason = kStopDP;
    }
}

// u <- t - (alpha_k / beta_k) u (u holds beta_k u_k); beta_{k+1} = ||u||. LSMR also
// forms A h_k = t - (theta_k / rho_{k-1}) A h_{k-1} in ah.
template <typename T>
__global__ __launch_bounds__(kBlock) void lsq_u_kernel(T *__restrict__ u, const T *__restrict__ t,
                                                       T *__restrict__ ah, long long m,
                                                       LsqScalars *S, double *partials,
                                                       unsigned *count, DevState *st, int k)
{
    __shared__ double lds[kWaves];
    __shared__ int last;
    if (halted(st, k)) return;
    const double cu = safe_div(S->alpha, S->beta);
    const double ch = safe_div(S->theta, S->rho_prev);
    double ss = 0.0;
    const long long T_ = (long long)gridDim.x * kBlock;
    for (long long l0 = (long long)blockIdx.x * kBlock + threadIdx.x; l0 < m; l0 += kLU * T_) {
        double tv[kLU], uv[kLU], hv[kLU];
#pragma unroll
        for (int j = 0; j < kLU; ++j) {
            const long long l = l0 + j * T_;
            const bool in = l < m;
            tv[j] = in ? to_f64(t[l]) : 0.0;
            uv[j] = in ? to_f64(u[l]) : 0.0;
            hv[j] = (in && ah) ? to_f64(ah[l]) : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kLU; ++j) {
            const long long l = l0 + j * T_;
            if (l >= m) continue;
            const double un = fma(-cu, uv[j], tv[j]);
            u[l] = (T)un;
            ss = fma(un, un, ss);
            if (ah) ah[l] = (T)fma(-ch, hv[j], tv[j]);
        }
    }
    double tot;
    if (last_block_total(ss, partials, count, lds, &tot, &last) && threadIdx.x == 0)
        S->beta_n = sqrt(tot);
}

// v <- s / beta_{k+1} - beta_{k+1} v (s = A^T u); alpha_{k+1} = ||v||.
template <typename T>
__global__ __launch_bounds__(kBlock) void lsq_v_kernel(T *__restrict__ v, const T *__restrict__ s,
                                                       long long n, LsqScalars *S, double *partials,
                                                       unsigned *count, DevState *st, int k)
{
    __shared__ double lds[kWaves];
    __shared__ int last;
    if (halted(st, k)) return;
    const double bn = S->beta_n;
    const double ib = safe_div(1.0, bn);
    double ss = 0.0;
    const long long T_ = (long long)gridDim.x * kBlock;
    for (long long l0 = (long long)blockIdx.x * kBlock + threadIdx.x; l0 < n; l0 += kLU * T_) {
        double sv[kLU], vv[kLU];
#pragma unroll
        for (int j = 0; j < kLU; ++j) {
            const long long l = l0 + j * T_;
            const bool in = l < n;
            sv[j] = in ? to_f64(s[l]) : 0.0;
            vv[j] = in ? to_f64(v[l]) : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kLU; ++j) {
            const long long l = l0 + j * T_;
            if (l >= n) continue;
            const double vn = fma(sv[j], ib, -bn * vv[j]);
            v[l] = (T)vn;
            ss = fma(vn, vn, ss);
        }
    }
    double tot;
    if (last_block_total(ss, partials, count, lds, &tot, &last) && threadIdx.x == 0)
        S->alpha_n = sqrt(tot);
}

// LSQR update of step k: rotation, x += (phi/rho) w, w <- v_{k+1} - (theta/rho) w,
// v_{k+1} = v / alpha_{k+1}; the last block stores the scalars, the residual estimate
// |phibar|, the DP candidate and the host copy of the scalars.
// xprev (optional): receives x_{k-1} (the NCP rule returns it when d_k > d_{k-1}).
template <typename T>
__global__ __launch_bounds__(kBlock) void lsqr_x_kernel(T *__restrict__ x, T *__restrict__ xprev,
                                                        T *__restrict__ w, T *__restrict__ v,
                                                        long long n, LsqScalars *S,
                                                        unsigned *count, DevState *st, int k,
                                                        DevState *snap)
{
    __shared__ int last;
    if (halted(st, k)) {
        if (snap && blockIdx.x == 0 && threadIdx.x == 0) *snap = *st;
        return;
    }
    const double bn = S->beta_n, an = S->alpha_n, rhobar = S->rhobar, phibar = S->phibar;
    const double rho = hypot(rhobar, bn);
    const double c = rho > 0.0 ? rhobar / rho : 1.0, sn = rho > 0.0 ? bn / rho : 0.0;
    const double theta = sn * an, phi = c * phibar;
    const double fx = safe_div(phi, rho), fw = safe_div(theta, rho), ia = safe_div(1.0, an);
    const long long T_ = (long long)gridDim.x * kBlock;
    for (long long l0 = (long long)blockIdx.x * kBlock + threadIdx.x; l0 < n; l0 += kLU * T_) {
        double wv[kLU], vv[kLU];
        T xv[kLU];
#pragma unroll
        for (int j = 0; j < kLU; ++j) {
            const long long l = l0 + j * T_;
            const bool in = l < n;
            wv[j] = in ? to_f64(w[l]) : 0.0;
            vv[j] = in ? to_f64(v[l]) : 0.0;
            xv[j] = in ? x[l] : T(0);
        }
#pragma unroll
        for (int j = 0; j < kLU; ++j) {
            const long long l = l0 + j * T_;
            if (l >= n) continue;
            const double vn = vv[j] * ia;
            if (xprev) xprev[l] = xv[j];
            x[l] = (T)fma(fx, wv[j], to_f64(xv[j]));
            w[l] = (T)fma(-fw, wv[j], vn);
            v[l] = (T)vn;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev = __hip_atomic_fetch_add(count, 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        last = prev == gridDim.x - 1;
    }
    __syncthreads();
    if (!last || threadIdx.x != 0) return;
    last_block_fence();
    __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    S->rhobar = -c * an;
    S->phibar = sn * phibar;
    S->alpha = an;
    S->beta = bn;
    st->res = fabs(sn * phibar);
    st->ls = fabs(sn * phibar * an * c);
    st->k = k;
    if (bn == 0.0 || an == 0.0) st->bd_k = k;
    dp_check(st, k);
    if (snap) *snap = *st;
}

// LSMR update of step k (rotations P_k and Pbar_k): hbar <- h - hcoef hbar,
// x += xcoef hbar, h <- v_{k+1} - (theta_{k+1}/rho_k) h, v_{k+1} = v / alpha_{k+1}; the
// last block stores the scalars (hcoef, xcoef for the residual kernel). xprev as for LSQR.
template <typename T>
__global__ __launch_bounds__(kBlock) void lsmr_x_kernel(T *__restrict__ x, T *__restrict__ xprev,
                                                        T *__restrict__ h, T *__restrict__ hbar,
                                                        T *__restrict__ v, long long n,
                                                        LsqScalars *S, unsigned *count,
                                                        DevState *st, int k)
{
    __shared__ int last;
    if (halted(st, k)) return;
    const double bn = S->beta_n, an = S->alpha_n;
    const double alphabar = S->alphabar, zetabar = S->zetabar;
    const double rho_prev = S->rho_prev, rhobar_prev = S->rhobar_prev;
    const double cbar = S->cbar, sbar = S->sbar;
    const double rho = hypot(alphabar, bn);
    const double c = rho > 0.0 ? alphabar / rho : 1.0, sn = rho > 0.0 ? bn / rho : 0.0;
    const double theta_n = sn * an, alphabar_n = c * an;
    const double thetabar = sbar * rho;
    const double rhobar = hypot(cbar * rho, theta_n);
    const double cbar_n = rhobar > 0.0 ? cbar * rho / rhobar : 1.0;
    const double sbar_n = rhobar > 0.0 ? theta_n / rhobar : 0.0;
    const double zeta = cbar_n * zetabar, zetabar_n = -sbar_n * zetabar;
    const double hcoef = safe_div(thetabar * rho, rho_prev * rhobar_prev);
    const double xcoef = safe_div(zeta, rho * rhobar);
    const double fh = safe_div(theta_n, rho), ia = safe_div(1.0, an);
    const long long T_ = (long long)gridDim.x * kBlock;
    for (long long l0 = (long long)blockIdx.x * kBlock + threadIdx.x; l0 < n; l0 += kLU * T_) {
        double hv[kLU], bv[kLU], vv[kLU];
        T xv[kLU];
#pragma unroll
        for (int j = 0; j < kLU; ++j) {
            const long long l = l0 + j * T_;
            const bool in = l < n;
            hv[j] = in ? to_f64(h[l]) : 0.0;
            bv[j] = in ? to_f64(hbar[l]) : 0.0;
            vv[j] = in ? to_f64(v[l]) : 0.0;
            xv[j] = in ? x[l] : T(0);
        }
#pragma unroll
        for (int j = 0; j < kLU; ++j) {
            const long long l = l0 + j * T_;
            if (l >= n) continue;
            const double hb = fma(-hcoef, bv[j], hv[j]);
            const double vn = vv[j] * ia;
            hbar[l] = (T)hb;
            if (xprev) xprev[l] = xv[j];
            x[l] = (T)fma(xcoef, hb, to_f64(xv[j]));
            h[l] = (T)fma(-fh, hv[j], vn);
            v[l] = (T)vn;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev = __hip_atomic_fetch_add(count, 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        last = prev == gridDim.x - 1;
    }
    __syncthreads();
    if (!last || threadIdx.x != 0) return;
    last_block_fence();
    __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    S->alphabar = alphabar_n;
    S->zetabar = zetabar_n;
    S->rho_prev = rho;
    S->rhobar_prev = rhobar;
    S->cbar = cbar_n;
    S->sbar = sbar_n;
    S->theta = theta_n;
    S->hcoef = hcoef;
    S->xcoef = xcoef;
    S->alpha = an;
    S->beta = bn;
    st->ls = fabs(zetabar_n);
    if (bn == 0.0 || an == 0.0) st->bd_k = k;
}

// LSMR residual of step k by recurrence: A hbar_k = A h_k - hcoef A hbar_{k-1},
// r_k = r_{k-1} - xcoef A hbar_k, ||r_k|| (DP candidate, host copy of the scalars).
template <typename T>
__global__ __launch_bounds__(kBlock) void lsmr_r_kernel(const T *__restrict__ ah, T *__restrict__ ahbar,
                                                        T *__restrict__ r, long long m, LsqScalars *S,
                                                        double *partials, unsigned *count,
                                                        DevState *st, int k, DevState *snap)
{
    __shared__ double lds[kWaves];
    __shared__ int last;
    if (halted(st, k)) {
        if (snap && blockIdx.x == 0 && threadIdx.x == 0) *snap = *st;
        return;
    }
    const double hcoef = S->hcoef, xcoef = S->xcoef;
    double ss = 0.0;
    const long long T_ = (long long)gridDim.x * kBlock;
    for (long long l0 = (long long)blockIdx.x * kBlock + threadIdx.x; l0 < m; l0 += kLU * T_) {
        double av[kLU], bv[kLU], rv[kLU];
#pragma unroll
        for (int j = 0; j < kLU; ++j) {
            const long long l = l0 + j * T_;
            const bool in = l < m;
            av[j] = in ? to_f64(ah[l]) : 0.0;
            bv[j] = in ? to_f64(ahbar[l]) : 0.0;
            rv[j] = in ? to_f64(r[l]) : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kLU; ++j) {
            const long long l = l0 + j * T_;
            if (l >= m) continue;
            const double hb = fma(-hcoef, bv[j], av[j]);
            const double rn = fma(-xcoef, hb, rv[j]);
            ahbar[l] = (T)hb;
            r[l] = (T)rn;
            ss = fma(rn, rn, ss);
        }
    }
    double tot;
    if (last_block_total(ss, partials, count, lds, &tot, &last) && threadIdx.x == 0) {
        st->res = sqrt(tot);
        st->k = k;
        dp_check(st, k);
        if (snap) *snap = *st;
    }
}

// After the first bidiagonalisation step (u = beta_1 u_1, v = alpha_1 v_1): v_1, the first
// search directions and the scalars; beta_1 = 0 (b - A x0 = 0) or alpha_1 = 0 (A^T r_0 = 0:
// x0 already minimises) stop at step 0.
template <typename T>
__global__ __launch_bounds__(kBlock) void lsq_start_kernel(T *__restrict__ v, T *__restrict__ w,
                                                           T *__restrict__ hbar, long long n,
                                                           LsqScalars *S, unsigned *count,
                                                           DevState *st, int lsmr)
{
    __shared__ int last;
    const double a1 = S->alpha_n, b1 = S->beta_n;
    const double ia = safe_div(1.0, a1);
    const long long T_ = (long long)gridDim.x * kBlock;
    for (long long l = (long long)blockIdx.x * kBlock + threadIdx.x; l < n; l += T_) {
        const double vn = to_f64(v[l]) * ia;
        v[l] = (T)vn;
        w[l] = (T)vn;                       // LSQR w_1 / LSMR h_1
        if (hbar) hbar[l] = (T)0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev = __hip_atomic_fetch_add(count, 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        last = prev == gridDim.x - 1;
    }
    __syncthreads();
    if (!last || threadIdx.x != 0) return;
    last_block_fence();
    __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    S->alpha = a1;
    S->beta = b1;
    S->rhobar = a1;
    S->phibar = b1;
    S->alphabar = a1;
    S->zetabar = a1 * b1;
    S->rho_prev = 1.0;
    S->rhobar_prev = 1.0;
    S->cbar = 1.0;
    S->sbar = 0.0;
    S->theta = 0.0;
    st->beta = b1;
    if (!isfinite(b1) || !isfinite(a1)) {
        st->error |= 2;
    } else if (b1 == 0.0 || a1 == 0.0) {
        st->stop = 1;
        st->stop_k = 0;
        st->stop_reason = kStopZero;
    }
    (void)lsmr;
}

// At most 256 blocks of kLU elements per thread and trip: the last block's final sum then
// reads one partial per thread.
unsigned blocks_of(long long L)
{
    long long b = (L + (long long)kBlock * kLU - 1) / ((long long)kBlock * kLU);
    return (unsigned)std::min<long long>(std::max<long long>(b, 1), 256);
}

}  // namespace

hipError_t launch_lsq_u(int t, void *u, const void *tv, void *ah, long long m, LsqScalars *S,
                        double *partials, unsigned *count, DevState *st, int k, hipStream_t s)
{
    if (t == ABG_F64)
        lsq_u_kernel<double><<<blocks_of(m), kBlock, 0, s>>>(
            static_cast<double *>(u), static_cast<const double *>(tv), static_cast<double *>(ah), m,
            S, partials, count, st, k);
    else
        lsq_u_kernel<float><<<blocks_of(m), kBlock, 0, s>>>(
            static_cast<float *>(u), static_cast<const float *>(tv), static_cast<float *>(ah), m, S,
            partials, count, st, k);
    return hipGetLastError();
}

hipError_t launch_lsq_v(int t, void *v, const void *sv, long long n, LsqScalars *S,
                        double *partials, unsigned *count, DevState *st, int k, hipStream_t s)
{
    if (t == ABG_F64)
        lsq_v_kernel<double><<<blocks_of(n), kBlock, 0, s>>>(
            static_cast<double *>(v), static_cast<const double *>(sv), n, S, partials, count, st, k);
    else
        lsq_v_kernel<float><<<blocks_of(n), kBlock, 0, s>>>(
            static_cast<float *>(v), static_cast<const float *>(sv), n, S, partials, count, st, k);
    return hipGetLastError();
}

hipError_t launch_lsqr_x(int t, void *x, void *xprev, void *w, void *v, long long n,
                         LsqScalars *S, unsigned *count, DevState *st, int k, DevState *snap,
                         hipStream_t s)
{
    if (t == ABG_F64)
        lsqr_x_kernel<double><<<blocks_of(n), kBlock, 0, s>>>(
            static_cast<double *>(x), static_cast<double *>(xprev), static_cast<double *>(w),
            static_cast<double *>(v), n, S, count, st, k, snap);
    else
        lsqr_x_kernel<float><<<blocks_of(n), kBlock, 0, s>>>(
            static_cast<float *>(x), static_cast<float *>(xprev), static_cast<float *>(w),
            static_cast<float *>(v), n, S, count, st, k, snap);
    return hipGetLastError();
}

hipError_t launch_lsmr_x(int t, void *x, void *xprev, void *h, void *hbar, void *v, long long n,
                         LsqScalars *S, unsigned *count, DevState *st, int k, hipStream_t s)
{
    if (t == ABG_F64)
        lsmr_x_kernel<double><<<blocks_of(n), kBlock, 0, s>>>(
            static_cast<double *>(x), static_cast<double *>(xprev), static_cast<double *>(h),
            static_cast<double *>(hbar), static_cast<double *>(v), n, S, count, st, k);
    else
        lsmr_x_kernel<float><<<blocks_of(n), kBlock, 0, s>>>(
            static_cast<float *>(x), static_cast<float *>(xprev), static_cast<float *>(h),
            static_cast<float *>(hbar), static_cast<float *>(v), n, S, count, st, k);
    return hipGetLastError();
}

hipError_t launch_lsmr_r(int t, const void *ah, void *ahbar, void *r, long long m, LsqScalars *S,
                         double *partials, unsigned *count, DevState *st, int k, DevState *snap,
                         hipStream_t s)
{
    if (t == ABG_F64)
        lsmr_r_kernel<double><<<blocks_of(m), kBlock, 0, s>>>(
            static_cast<const double *>(ah), static_cast<double *>(ahbar), static_cast<double *>(r), m,
            S, partials, count, st, k, snap);
    else
        lsmr_r_kernel<float><<<blocks_of(m), kBlock, 0, s>>>(
            static_cast<const float *>(ah), static_cast<float *>(ahbar), static_cast<float *>(r), m, S,
            partials, count, st, k, snap);
    return hipGetLastError();
}

hipError_t launch_lsq_start(int t, void *v, void *w, void *hbar, long long n, LsqScalars *S,
                            unsigned *count, DevState *st, int lsmr, hipStream_t s)
{
    if (t == ABG_F64)
        lsq_start_kernel<double><<<blocks_of(n), kBlock, 0, s>>>(
            static_cast<double *>(v), static_cast<double *>(w), static_cast<double *>(hbar), n, S, count,
            st, lsmr);
    else
        lsq_start_kernel<float><<<blocks_of(n), kBlock, 0, s>>>(
            static_cast<float *>(v), static_cast<float *>(w), static_cast<float *>(hbar), n, S, count, st,
            lsmr);
    return hipGetLastError();
}

}  // namespace abg
