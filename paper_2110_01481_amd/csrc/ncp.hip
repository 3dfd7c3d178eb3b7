// NCP stopping criterion (Sec. 6.3) on gfx950.
//
// For each sinogram row of the residual: the periodogram
// p_j = |DFT_j|^2, j = 1..q = floor(n_det/2), then the normalised cumulative sum
// c(j) = sum_{l<=j} p_l / sum_{l<=q} p_l. Two more kernels average c over the rows per j
// (column sums over chunks of rows, then the chunks in order) and form the distance to
// the white-noise line j/q.
//
// The DFT of a row of any length n (2897 at the largest scan is prime) is taken with
// Bluestein's chirp transform: with c_i = exp(-pi i i^2/n), 2ij = i^2 + j^2 - (j-i)^2
// gives X_j = c_j sum_i (r_i c_i) conj(c_{j-i}), a linear convolution of length 2n-1,
// done cyclically with two power-of-two FFTs of length M >= 2n-1 held in LDS (M <= 8192:
// 128 KB of complex FP64, 144 KB with one padding slot per eight). One block transforms
// two rows at once, packed as the real and imaginary part of one complex row (the rows are
// real; their spectra are separated by conjugate symmetry after the final chirp); the 1/M
// of the inverse transform cancels in the normalisation. The
// transform of the fixed chirp kernel conj(c_t), the chirp c_i and the twiddle factors
// are computed once per geometry on the host (FP64) and kept on the device. Short rows
// (n < 64) and rows too long for LDS use Goertzel's recurrence per frequency instead
// (O(n) work per frequency, FP64).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <mutex>
#include <vector>

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

// Column sums of crow over chunks of rows: block (jb, c) adds rows c*rows_per .. of
// frequencies jb*kBlock + t into colsum[c][j] (many blocks, short loops: the rows of a
// scan are read once, spread over the device).
constexpr int kRowChunks = 32;

__global__ __launch_bounds__(kBlock) void ncp_colsum_kernel(const double *__restrict__ crow,
                                                            int n_ang, int q, int rows_per,
                                                            double *__restrict__ colsum,
                                                            const DevState *st, int k)
{
    if (halted(st, k)) return;
    const int j = blockIdx.x * kBlock + threadIdx.x;
    const int a0 = blockIdx.y * rows_per, a1 = min(n_ang, a0 + rows_per);
    if (j >= q) return;
    // in row order, eight rows' loads issued before their adds
    double s = 0.0;
    int a = a0;
    for (; a + 8 <= a1; a += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = crow[(size_t)(a + u) * q + j];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; a < a1; ++a) s += crow[(size_t)a * q + j];
    colsum[(size_t)blockIdx.y * q + j] = s;
}

// (mean over rows - j/q)^2 per frequency, the chunks' sums added in chunk order; one
// partial per block.
__global__ __launch_bounds__(kBlock) void ncp_dist_kernel(const double *__restrict__ colsum,
                                                          int n_chunks, int n_ang, int q,
                                                          double *__restrict__ partials,
                                                          const DevState *st, int k)
{
    __shared__ double lds[kBlock / 64];
    if (halted(st, k)) return;
    const int j = blockIdx.x * kBlock + threadIdx.x;
    double d2 = 0.0;
    if (j < q) {
        double s = 0.0;
        int c = 0;
        for (; c + 8 <= n_chunks; c += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = colsum[(size_t)(c + u) * q + j];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; c < n_chunks; ++c) s += colsum[(size_t)c * q + j];
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

// ---- Bluestein rows: forward FFT (decimation in frequency: natural order in, bit-
// reversed order out), product with the kernel's transform (stored bit-reversed), inverse
// FFT (decimation in time: bit-reversed in, natural out) -- no permutation pass.
constexpr int kFftThreads = 1024;
constexpr int kFftMaxM = 8192;

__device__ inline double2 cmul(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

// Rows 2b and 2b + 1 of the sinogram share one complex transform: z = (x_a + i x_b) c,
// and the DFT Z = c * conv of that packed row gives both rows' spectra by conjugate
// symmetry (the rows are real): X_a[j] = (Z[j] + conj(Z[n-j])) / 2 and
// X_b[j] = (Z[j] - conj(Z[n-j])) / 2i. Adjacent angles are paired, so the two rows have
// similar magnitudes and each row's share of the rounding stays at its own level. A row
// that is zero everywhere takes the white-noise line j/q, as in the one-row definition
// (its packed spectrum would be the other row's rounding).
template <typename T>
__global__ __launch_bounds__(kFftThreads) void ncp_fft_rows_kernel(
    const T *__restrict__ r, int n_ang, int n_det, int q, int M, const double2 *__restrict__ chirp,
    const double2 *__restrict__ khat, const double2 *__restrict__ tw, double *__restrict__ crow,
    const DevState *st, int k)
{
    extern __shared__ double2 zs[];         // M values in M + M / 8 slots
    __shared__ double wsum[2][kFftThreads / 64];
    __shared__ double total_s[2];
    if (halted(st, k)) return;
    // element i at i + i / 8: a lane's run of 4 or 8 consecutive elements (the passes of
    // short spans) and runs of consecutive lanes both spread over the LDS banks
    auto z = [&](int i) -> double2 & { return zs[i + (i >> 3)]; };
    const int t = threadIdx.x;
    const int ra = 2 * (int)blockIdx.x, rb = ra + 1;
    const bool has_b = rb < n_ang;
    const T *src_a = r + (size_t)ra * n_det;
    const T *src_b = r + (size_t)(has_b ? rb : ra) * n_det;
    // all of a thread's loads issued before the first is used (M / kFftThreads <= 8)
    int nz_a = 0, nz_b = 0;
    {
        constexpr int kPer = kFftMaxM / kFftThreads;
        double xa[kPer], xb[kPer];
        double2 c[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int i = t + u * kFftThreads;
            const bool in = i < n_det;
            xa[u] = in ? (double)src_a[i] : 0.0;
            xb[u] = in && has_b ? (double)src_b[i] : 0.0;
            c[u] = in ? chirp[i] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int i = t + u * kFftThreads;
            nz_a |= xa[u] != 0.0;
            nz_b |= xb[u] != 0.0;
            if (i < M) z(i) = cmul(make_double2(xa[u], xb[u]), c[u]);
        }
    }
    const bool live_a = __syncthreads_or(nz_a) != 0;
    const bool live_b = __syncthreads_or(nz_b) != 0;
    const int half = M >> 1, quarter = M >> 2;
    // Radix-2 butterflies. Decimation in frequency, span h: (u, v) -> (u + v, (u - v) w);
    // decimation in time: (u, v) -> (u + v conj(w), u - v conj(w)); w = exp(-2 pi i j /
    // (2h)) = tw[h - 1 + j] for the pair's offset j < h in its block of 2h (a pass's
    // twiddles are contiguous: adjacent lanes read adjacent entries).
    auto dif = [](double2 &u, double2 &v, double2 w) {
        const double dx = u.x - v.x, dy = u.y - v.y;
        u = make_double2(u.x + v.x, u.y + v.y);
        v = make_double2(fma(dx, w.x, -dy * w.y), fma(dx, w.y, dy * w.x));
    };
    auto dit = [](double2 &u, double2 &v, double2 w) {
        const double px = fma(v.x, w.x, v.y * w.y), py = fma(v.y, w.x, -v.x * w.y);
        v = make_double2(u.x - px, u.y - py);
        u = make_double2(u.x + px, u.y + py);
    };
    // Two or three consecutive passes run as one: a thread takes the 4 (8) elements that
    // the spans join (offsets j + m g of a block of 4g (8g)) through the passes in
    // registers -- the same operations on every element as the radix-2 passes, with a
    // half (a third) of the LDS traffic and barriers. The product with the kernel's
    // transform is taken in the loads of the inverse transform's first pass (span 1).
    int lg = 0;
    while ((1 << lg) < M) ++lg;
    const int eighth = M >> 3;
    auto pass1 = [&](int h, bool inv) {                 // span h alone
        for (int b = t; b < half; b += kFftThreads) {
            const int j = b & (h - 1), i = ((b - j) << 1) + j;
            double2 u = z(i), v = z(i + h);
            if (inv) {
                if (h == 1) {
                    u = cmul(u, khat[i]);
                    v = cmul(v, khat[i + 1]);
                }
                dit(u, v, tw[h - 1 + j]);
            } else {
                dif(u, v, tw[h - 1 + j]);
            }
            z(i) = u;
            z(i + h) = v;
        }
        __syncthreads();
    };
    auto pass2 = [&](int g, bool inv) {                 // spans 2g, g (forward); g, 2g
        for (int b = t; b < quarter; b += kFftThreads) {
            const int j = b & (g - 1), i = ((b - j) << 2) + j;
            double2 a0 = z(i), a1 = z(i + g), a2 = z(i + 2 * g), a3 = z(i + 3 * g);
            if (inv) {
                if (g == 1) {
                    a0 = cmul(a0, khat[i]);
                    a1 = cmul(a1, khat[i + 1]);
                    a2 = cmul(a2, khat[i + 2]);
                    a3 = cmul(a3, khat[i + 3]);
                }
                const double2 w1 = tw[g - 1 + j];
                dit(a0, a1, w1);
                dit(a2, a3, w1);
                dit(a0, a2, tw[2 * g - 1 + j]);
                dit(a1, a3, tw[2 * g - 1 + j + g]);
            } else {
                dif(a0, a2, tw[2 * g - 1 + j]);
                dif(a1, a3, tw[2 * g - 1 + j + g]);
                const double2 w1 = tw[g - 1 + j];
                dif(a0, a1, w1);
                dif(a2, a3, w1);
            }
            z(i) = a0;
            z(i + g) = a1;
            z(i + 2 * g) = a2;
            z(i + 3 * g) = a3;
        }
        __syncthreads();
    };
    auto pass3 = [&](int g, bool inv) {                 // spans 4g, 2g, g; g, 2g, 4g
        for (int b = t; b < eighth; b += kFftThreads) {
            const int j = b & (g - 1), i = ((b - j) << 3) + j;
            double2 a[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) a[m] = z(i + m * g);
            const double2 w2a = tw[2 * g - 1 + j], w2b = tw[2 * g - 1 + j + g];
            const double2 w1 = tw[g - 1 + j];
            if (inv) {
                if (g == 1) {
#pragma unroll
                    for (int m = 0; m < 8; ++m) a[m] = cmul(a[m], khat[i + m]);
                }
#pragma unroll
                for (int m = 0; m < 8; m += 2) dit(a[m], a[m + 1], w1);
                dit(a[0], a[2], w2a);
                dit(a[1], a[3], w2b);
                dit(a[4], a[6], w2a);
                dit(a[5], a[7], w2b);
#pragma unroll
                for (int m = 0; m < 4; ++m) dit(a[m], a[m + 4], tw[4 * g - 1 + j + m * g]);
            } else {
#pragma unroll
                for (int m = 0; m < 4; ++m) dif(a[m], a[m + 4], tw[4 * g - 1 + j + m * g]);
                dif(a[0], a[2], w2a);
                dif(a[1], a[3], w2b);
                dif(a[4], a[6], w2a);
                dif(a[5], a[7], w2b);
#pragma unroll
                for (int m = 0; m < 8; m += 2) dif(a[m], a[m + 1], w1);
            }
#pragma unroll
            for (int m = 0; m < 8; ++m) z(i + m * g) = a[m];
        }
        __syncthreads();
    };
    // forward: spans M/2 .. 1, the lg mod 3 largest first
    int h = half;
    if (lg % 3 == 1) {
        pass1(h, false);
        h >>= 1;
    } else if (lg % 3 == 2) {
        pass2(h >> 1, false);
        h >>= 2;
    }
    for (; h >= 4; h >>= 3) pass3(h >> 2, false);
    // inverse: spans 1 .. M/2, the lg mod 3 largest last
    for (h = 1; 8 * h <= M; h <<= 3) pass3(h, true);
    if (lg % 3 == 1) pass1(h, true);
    else if (lg % 3 == 2) pass2(h, true);
    // both rows' periodograms at frequency j (up to the common factor M^2 / 4)
    auto power = [&](int j, double &pa, double &pb) {
        const double2 zj = cmul(z(j), chirp[j]);
        const double2 zn = cmul(z(n_det - j), chirp[n_det - j]);
        const double ax = zj.x + zn.x, ay = zj.y - zn.y;    // 2 X_a
        const double bx = zj.y + zn.y, by = zn.x - zj.x;    // 2 X_b
        pa = fma(ax, ax, ay * ay);
        pb = fma(bx, bx, by * by);
    };
    // thread t owns frequencies j = 1 + t*J .. (t+1)*J (J <= 2, as q <= (M + 1) / 4);
    // their powers are formed once, with every load issued up front (a frequency past the
    // thread's share reads frequency q and is dropped); fixed-order prefix over threads
    constexpr int kMaxJ = (kFftMaxM / 4 + kFftThreads - 1) / kFftThreads;
    const int J = (q + kFftThreads - 1) / kFftThreads;
    double own_a = 0.0, own_b = 0.0;
    double pa[kMaxJ], pb[kMaxJ];
#pragma unroll
    for (int u = 0; u < kMaxJ; ++u) power(min(1 + t * J + u, q), pa[u], pb[u]);
#pragma unroll
    for (int u = 0; u < kMaxJ; ++u) {
        if (u < J && 1 + t * J + u <= q) {
            own_a += pa[u];
            own_b += pb[u];
        }
    }
    // inclusive scans within the wave, then wave totals in order
    const int lane = t & 63, wv = t >> 6;
    double inc_a = own_a, inc_b = own_b;
    for (int o = 1; o < 64; o <<= 1) {
        const double na = __shfl_up(inc_a, o, 64), nb = __shfl_up(inc_b, o, 64);
        if (lane >= o) {
            inc_a += na;
            inc_b += nb;
        }
    }
    if (lane == 63) {
        wsum[0][wv] = inc_a;
        wsum[1][wv] = inc_b;
    }
    __syncthreads();
    if (t < 2) {
        double run = 0.0;
        for (int w = 0; w < kFftThreads / 64; ++w) {
            const double v = wsum[t][w];
            wsum[t][w] = run;
            run += v;
        }
        total_s[t] = run;
    }
    __syncthreads();
    const double total_a = live_a ? total_s[0] : 0.0, total_b = live_b ? total_s[1] : 0.0;
    double acc_a = wsum[0][wv] + inc_a - own_a, acc_b = wsum[1][wv] + inc_b - own_b;
#pragma unroll
    for (int u = 0; u < kMaxJ; ++u) {
        const int j = 1 + t * J + u;
        if (u < J && j <= q) {
            acc_a += pa[u];
            acc_b += pb[u];
            const double white = (double)j / (double)q;
            crow[(size_t)ra * q + (j - 1)] = total_a > 0.0 ? acc_a / total_a : white;
            if (has_b) crow[(size_t)rb * q + (j - 1)] = total_b > 0.0 ? acc_b / total_b : white;
        }
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

int fft_length(int n_det)
{
    if (n_det < 64) return 0;
    int M = 1;
    while (M < 2 * n_det - 1) M <<= 1;
    return M <= kFftMaxM ? M : 0;
}

// Host FFT (FP64, radix 2, decimation in time after a bit-reversal permutation) of the
// chirp kernel; the same twiddles as the device.
void host_fft(std::vector<std::complex<double>> &a, const std::vector<std::complex<double>> &tw)
{
    const int M = (int)a.size();
    for (int i = 1, j = 0; i < M; ++i) {
        int bit = M >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (int h = 1; h < M; h <<= 1)
        for (int i0 = 0; i0 < M; i0 += 2 * h)
            for (int j = 0; j < h; ++j) {
                const std::complex<double> v = a[i0 + j + h] * tw[(size_t)j * (M / (2 * h))];
                a[i0 + j + h] = a[i0 + j] - v;
                a[i0 + j] += v;
            }
}

std::mutex g_ncp_mu;
std::atomic<int> g_force_goertzel{0};

// Chirp (n), kernel transform in bit-reversed order (M) and the twiddles of every pass
// (M - 1: the pass of span h holds exp(-2 pi i j / (2h)), j < h, at h - 1 + j) of the
// geometry's row length, built on first use and kept with the geometry.
hipError_t ncp_tables(const Geometry &g, int M, const double2 **chirp, const double2 **khat,
                      const double2 **tw)
{
    std::lock_guard<std::mutex> lk(g_ncp_mu);
    const int n = g.n_det;
    if (!g.ncp_tab) {
        const double pi = 3.14159265358979323846;
        std::vector<std::complex<double>> c(n), w(M / 2), kern(M, 0.0);
        for (int i = 0; i < n; ++i) {
            const long long e = ((long long)i * i) % (2LL * n);   // c_i = exp(-pi i e / n)
            c[i] = std::polar(1.0, -pi * (double)e / (double)n);
        }
        for (int j = 0; j < M / 2; ++j) w[j] = std::polar(1.0, -2.0 * pi * (double)j / (double)M);
        kern[0] = std::conj(c[0]);
        for (int i = 1; i < n; ++i) kern[i] = kern[M - i] = std::conj(c[i]);
        host_fft(kern, w);
        std::vector<double2> tab((size_t)n + 2 * M - 1);
        for (int i = 0; i < n; ++i) tab[i] = make_double2(c[i].real(), c[i].imag());
        const int bits = __builtin_ctz(M);
        for (int i = 0; i < M; ++i) {
            const unsigned br = __builtin_bitreverse32((unsigned)i) >> (32 - bits);
            tab[(size_t)n + i] = make_double2(kern[br].real(), kern[br].imag());
        }
        for (int h = 1; h < M; h <<= 1)
            for (int j = 0; j < h; ++j) {
                // exp(-2 pi i j / (2h)) = w[j M / (2h)]
                const std::complex<double> v = w[(size_t)j * (M / (2 * h))];
                tab[(size_t)n + M + h - 1 + j] = make_double2(v.real(), v.imag());
            }
        void *d = nullptr;
        hipError_t e = hipMalloc(&d, tab.size() * sizeof(double2));
        if (e != hipSuccess) return e;
        e = hipMemcpy(d, tab.data(), tab.size() * sizeof(double2), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            return e;
        }
        g.ncp_tab = d;
    }
    const double2 *base = static_cast<const double2 *>(g.ncp_tab);
    *chirp = base;
    *khat = base + n;
    *tw = base + n + M;
    return hipSuccess;
}

template <typename T>
hipError_t fft_rows_go(const Geometry &g, int M, const void *r, double *crow, int q,
                       const DevState *st, int k, hipStream_t s)
{
    const double2 *chirp, *khat, *tw;
    hipError_t e = ncp_tables(g, M, &chirp, &khat, &tw);
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)(M + M / 8) * sizeof(double2);   // skewed: one slot per eight
    ncp_fft_rows_kernel<T><<<(g.n_ang + 1) / 2, kFftThreads, lds, s>>>(
        static_cast<const T *>(r), g.n_ang, g.n_det, q, M, chirp, khat, tw, crow, st, k);
    return hipGetLastError();
}

}  // namespace

void ncp_force_goertzel(int on) { g_force_goertzel.store(on ? 1 : 0); }

void ncp_release(Geometry &g)
{
    if (g.ncp_tab) (void)hipFree(g.ncp_tab);
    g.ncp_tab = nullptr;
}

size_t ncp_scratch_bytes(const Geometry &g)
{
    const int q = g.n_det / 2;
    const size_t nb = (size_t)(q + kBlock - 1) / kBlock;
    return align256((size_t)g.n_ang * q * sizeof(double)) +
           align256((size_t)kRowChunks * q * sizeof(double)) + align256((nb + 1) * sizeof(double));
}

hipError_t launch_ncp(const Geometry &g, int t, const void *r, double *scratch, DevState *st,
                      int k, hipStream_t s, DevState *snap)
{
    const int q = g.n_det / 2;
    if (q < 1) return hipErrorInvalidValue;
    double *crow = scratch;
    double *colsum = crow + align256((size_t)g.n_ang * q * sizeof(double)) / sizeof(double);
    double *part = colsum + align256((size_t)kRowChunks * q * sizeof(double)) / sizeof(double);
    // timed from before the row kernel to after the final one when profiling is on
    const int M = g_force_goertzel.load() ? 0 : fft_length(g.n_det);
    // tables first: building them (once per geometry) must not fall inside the timing
    if (M) {
        const double2 *c, *kh, *tw;
        hipError_t e = ncp_tables(g, M, &c, &kh, &tw);
        if (e != hipSuccess) return e;
    }
    ProfScope ps(kProfNcp, s, st ? k : 0, false);
    hipError_t e = M ? (t == ABG_F64 ? fft_rows_go<double>(g, M, r, crow, q, st, k, s)
                                     : fft_rows_go<float>(g, M, r, crow, q, st, k, s))
                     : (t == ABG_F64 ? rows_dispatch<double>(g, r, crow, q, st, k, s)
                                     : rows_dispatch<float>(g, r, crow, q, st, k, s));
    if (e != hipSuccess) return e;
    const int nb = (q + kBlock - 1) / kBlock;
    const int chunks = std::min(kRowChunks, g.n_ang);
    const int rows_per = (g.n_ang + chunks - 1) / chunks;
    ncp_colsum_kernel<<<dim3(nb, chunks), kBlock, 0, s>>>(crow, g.n_ang, q, rows_per, colsum, st, k);
    ncp_dist_kernel<<<nb, kBlock, 0, s>>>(colsum, chunks, g.n_ang, q, part, st, k);
    ncp_final_kernel<<<1, 64, 0, s>>>(part, nb, st, k, snap);
    return hipGetLastError();
}

}  // namespace abg
