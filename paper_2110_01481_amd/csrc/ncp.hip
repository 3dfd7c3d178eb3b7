// NCP stopping criterion (Sec. 6.3) on gfx950.
//
// For each sinogram row of the residual (one block per row): the periodogram
// p_j = |DFT_j|^2, j = 1..q = floor(n_det/2), by Goertzel's second-order recurrence in
// FP64 (one recurrence per frequency, no twiddle table; n_det may be prime), then the
// normalised cumulative sum c(j) = sum_{l<=j} p_l / sum_{l<=q} p_l. A second kernel
// averages c over the rows per j and forms the distance to the white-noise line j/q.
#include <cmath>

#include "abg_internal.h"

namespace abg {
namespace {

constexpr int kBlock = 256;

template <typename T, int J>
__global__ __launch_bounds__(kBlock) void ncp_rows_kernel(const T *__restrict__ r, int n_det,
                                                          int q, double *__restrict__ crow,
                                                          const DevState *st, int k)
{
    extern __shared__ double row[];
    __shared__ double chunk[kBlock];
    if (halted(st, k)) return;
    const int a = blockIdx.x;
    const T *src = r + (size_t)a * n_det;
    for (int i = threadIdx.x; i < n_det; i += kBlock) row[i] = (double)src[i];
    __syncthreads();
    // thread t owns frequencies j = 1 + t*J .. t*J + J
    double cf[J], s1[J], s2[J];
#pragma unroll
    for (int u = 0; u < J; ++u) {
        const int j = 1 + threadIdx.x * J + u;
        cf[u] = 2.0 * cospi(2.0 * (double)j / (double)n_det);
        s1[u] = 0.0;
        s2[u] = 0.0;
    }
    for (int i = 0; i < n_det; ++i) {
        const double v = row[i];
#pragma unroll
        for (int u = 0; u < J; ++u) {
            const double s0 = fma(cf[u], s1[u], v - s2[u]);
            s2[u] = s1[u];
            s1[u] = s0;
        }
    }
    double p[J];
    double tot = 0.0;
#pragma unroll
    for (int u = 0; u < J; ++u) {
        const int j = 1 + threadIdx.x * J + u;
        // |X_j|^2 = s1^2 + s2^2 - 2cos(w) s1 s2 with s1 = s_{n-1}, s2 = s_{n-2}
        p[u] = (j <= q) ? fma(s1[u], s1[u], fma(s2[u], s2[u], -cf[u] * s1[u] * s2[u])) : 0.0;
        tot += p[u];
    }
    chunk[threadIdx.x] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        double run = 0.0;
        for (int t = 0; t < kBlock; ++t) {
            const double v = chunk[t];
            chunk[t] = run;   // exclusive prefix, fixed order
            run += v;
        }
        row[0] = run;         // row values are no longer needed; keep the total here
    }
    __syncthreads();
    const double total = row[0];
    double acc = chunk[threadIdx.x];
#pragma unroll
    for (int u = 0; u < J; ++u) {
        const int j = 1 + threadIdx.x * J + u;
        if (j <= q) {
            acc += p[u];
            crow[(size_t)a * q + (j - 1)] = total > 0.0 ? acc / total : (double)j / (double)q;
        }
    }
}

__global__ __launch_bounds__(kBlock) void ncp_mean_kernel(const double *__restrict__ crow, int n_ang,
                                                          int q, double *__restrict__ partials,
                                                          const DevState *st, int k)
{
    __shared__ double lds[kBlock / 64];
    if (halted(st, k)) return;
    const int j = blockIdx.x * kBlock + threadIdx.x;
    double d2 = 0.0;
    if (j < q) {
        double s = 0.0;
        for (int a = 0; a < n_ang; ++a) s += crow[(size_t)a * q + j];
        const double dev = s / (double)n_ang - (double)(j + 1) / (double)q;
        d2 = dev * dev;
    }
    for (int o = 32; o > 0; o >>= 1) d2 += __shfl_xor(d2, o, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = d2;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += lds[w];
        partials[blockIdx.x] = t;
    }
}

// d_k = sqrt(sum of partials); the NCP stop is raised at the first k >= 2 whose d_k
// exceeds d_{k-1} (the iterate to return is then x_{k-1}).
__global__ void ncp_final_kernel(const double *partials, int nb, DevState *st, int k,
                                 DevState *snap)
{
    if (halted(st, k)) {
        if (snap && threadIdx.x == 0 && blockIdx.x == 0) *snap = *st;
        return;
    }
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double t = 0.0;
        for (int b = 0; b < nb; ++b) t += partials[b];
        const double d = sqrt(t);
        st->ncp = d;
        if (!isfinite(d)) {
            st->error |= 2;
        } else if (k >= 2 && d > st->ncp_prev && !st->stop) {
            st->stop = 1;
            st->stop_k = k;
            st->stop_reason = kStopNCP;
        }
        st->ncp_prev = d;
        if (snap) *snap = *st;
    }
}

template <typename T, int J>
hipError_t rows_go(const Geometry &g, const void *r, double *crow, int q, const DevState *st,
                   int k, hipStream_t s)
{
    const size_t lds = (size_t)g.n_det * sizeof(double);
    ncp_rows_kernel<T, J><<<g.n_ang, kBlock, lds, s>>>(static_cast<const T *>(r), g.n_det, q, crow,
                                                       st, k);
    return hipGetLastError();
}

template <typename T>
hipError_t rows_dispatch(const Geometry &g, const void *r, double *crow, int q,
                         const DevState *st, int k, hipStream_t s)
{
    if (q <= kBlock) return rows_go<T, 1>(g, r, crow, q, st, k, s);
    if (q <= 2 * kBlock) return rows_go<T, 2>(g, r, crow, q, st, k, s);
    if (q <= 4 * kBlock) return rows_go<T, 4>(g, r, crow, q, st, k, s);
    if (q <= 8 * kBlock) return rows_go<T, 8>(g, r, crow, q, st, k, s);
    return hipErrorInvalidValue;
}

}  // namespace

size_t ncp_scratch_bytes(const Geometry &g)
{
    const int q = g.n_det / 2;
    const size_t nb = (size_t)(q + kBlock - 1) / kBlock;
    return align256((size_t)g.n_ang * q * sizeof(double)) + align256((nb + 1) * sizeof(double));
}

hipError_t launch_ncp(const Geometry &g, int t, const void *r, double *scratch, DevState *st,
                      int k, hipStream_t s, DevState *snap)
{
    const int q = g.n_det / 2;
    if (q < 1) return hipErrorInvalidValue;
    double *crow = scratch;
    double *part = scratch + align256((size_t)g.n_ang * q * sizeof(double)) / sizeof(double);
    // timed from before the row kernel to after the final one when profiling is on
    ProfScope ps(kProfNcp, s, st ? k : 0, false);
    hipError_t e = t == ABG_F64 ? rows_dispatch<double>(g, r, crow, q, st, k, s)
                                : rows_dispatch<float>(g, r, crow, q, st, k, s);
    if (e != hipSuccess) return e;
    const int nb = (q + kBlock - 1) / kBlock;
    ncp_mean_kernel<<<nb, kBlock, 0, s>>>(crow, g.n_ang, q, part, st, k);
    ncp_final_kernel<<<1, 64, 0, s>>>(part, nb, st, k, snap);
    return hipGetLastError();
}

}  // namespace abg
