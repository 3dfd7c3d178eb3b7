// Device code of the ray-driven forward projector (line model), shared by the
// single-problem kernels (projectors.hip) and the batched kernels (batch.hip), so that
// both run the same arithmetic.
#pragma once

#include <cmath>

#include "abg_internal.h"

namespace abg {
namespace {

constexpr int kFwdBlock = 256;
// An axis-aligned ray lies on a pixel edge when its offset from the edge is below this
// (in pixels): bin positions carry rounding error, and an edge ray in exact arithmetic
// must split evenly.
constexpr double kEdgeTie = 1e-9;

__device__ inline int wave_min_i(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline int wave_max_i(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Writes the zero-padded row-major copy xr (N x S, image column c at c + kPad) and the
// transposed copy xc (row c of xc = column c of the image), through a 32 x 33 LDS tile.
template <typename T> struct PadLds {
    T tile[32][33];
};
template <typename T>
__device__ inline void pad_transpose_tile(const T *__restrict__ x, T *__restrict__ xr,
                                          T *__restrict__ xc, int N, int S, int bx, int by,
                                          PadLds<T> &lds)
{
    T (*tile)[33] = lds.tile;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int j = ty; j < 32; j += 8) {
        const int r = by + j, c = bx + tx;
        T v = T(0);
        if (r < N && c < N) {
            v = x[(size_t)r * N + c];
            xr[(size_t)r * S + c + kPad] = v;
        }
        tile[j][tx] = v;
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int c = bx + j, r = by + tx;
        if (c < N && r < N) xc[(size_t)c * S + r + kPad] = tile[tx][j];
    }
}

// Zeroes the kPad columns on both sides of the 2N padded rows of xr and xc.
template <typename T>
__device__ inline void pad_zero_item(T *__restrict__ xr, T *__restrict__ xc, int N, int S, int idx)
{
    const int per_row = 2 * kPad;
    if (idx >= 2 * N * per_row) return;
    const int row = idx / per_row, e = idx % per_row;
    const int col = e < kPad ? e : N + e;   // [0,kPad) and [N+kPad, N+2kPad)
    T *base = row < N ? xr + (size_t)row * S : xc + (size_t)(row - N) * S;
    base[col] = T(0);
}

// Position of a ray inside the current band of pixels: the band holds the minor-axis
// interval [lo, lo + |m|] (pixels from the image edge) and the walk advances lo by m.
// FP64 data: lo in FP64. FP32 data: lo biased by kPad as an integer column and a 32-bit
// fraction, so a band step is an add with carry, the pixel index is the integer part and
// the fraction gives the weight.
template <typename T> struct Band;
template <typename T> struct BandWeights {
    T invq, len;
    __device__ BandWeights(double iq, double l) : invq(T(iq)), len(T(l)) {}
};

template <> struct Band<double> {
    double lo, m;
    __device__ Band(double lo0, double m_) : lo(lo0), m(m_) {}
    __device__ void next() { lo += m; }
    __device__ unsigned column(unsigned cmax) const
    {
        return min((unsigned)((int)floor(lo) + kPad), cmax);
    }
    // length of the band segment left of the pixel edge at floor(lo) + 1
    __device__ double left_length(const BandWeights<double> &b) const
    {
        return fmin(b.len, fma(floor(lo) - lo, b.invq, b.invq));
    }
};

template <> struct Band<float> {
    // lo + kPad = c + f / 2^32: integer column and 32-bit fraction, stepped by the split
    // slope (mi, mf) with one add and one add-with-carry; error < 1e-6 px after 2^12 steps
    int c;
    unsigned f;
    int mi;
    unsigned mf;
    __device__ Band(double lo0, double m)
    {
        const double p = lo0 + kPad;
        const double pc = floor(p);
        c = (int)pc;
        f = (unsigned)min(__double2ull_rn((p - pc) * 0x1p32), 0xffffffffull);
        const double mc = floor(m);
        mi = (int)mc;
        mf = (unsigned)min(__double2ull_rn((m - mc) * 0x1p32), 0xffffffffull);
    }
    __device__ void next()
    {
        const unsigned nf = f + mf;
        c += mi + (nf < f ? 1 : 0);
        f = nf;
    }
    __device__ unsigned column(unsigned cmax) const
    {
        return (unsigned)min(max(c, 0), (int)cmax);
    }
    __device__ float left_length(const BandWeights<float> &b) const
    {
        const float w = fmaf((float)f, -b.invq * 0x1p-32f, b.invq);
        return __builtin_amdgcn_fmed3f(w, b.len, -1e30f);   // min(w, len)
    }
};

// The two adjacent pixels a band segment can touch, fetched with one load from a
// wave-uniform row pointer plus a 32-bit byte offset (one wide gather is cheaper for
// the texture address unit than two narrow ones).
template <typename T> struct alignas(sizeof(T)) Taps {
    T a, b;
};
template <typename T>
__device__ inline Taps<T> load_taps(const T *row, unsigned col)
{
    const unsigned boff = col * (unsigned)sizeof(T);
    return *reinterpret_cast<const Taps<T> *>(reinterpret_cast<const char *>(row) + boff);
}

// Ray i of angle a (i may exceed n_det: such lanes only take part in the wave's band
// range and store nothing). Called by whole waves of consecutive rays.
template <typename T>
__device__ inline void forward_ray(const T *__restrict__ xr, const T *__restrict__ xc,
                                   T *__restrict__ y, const AngleParams *__restrict__ ang, int a,
                                   int i, int N, int S, int n_det, double ds, double s0)
{
    const AngleParams P = ang[a];
    const T *img = (P.steep ? xr : xc) + kPad;
    const double half = 0.5 * N;
    const double si = s0 + (double)i * ds;
    // minor-axis coordinate, in pixels from the image edge, where the ray enters band 0
    const double u0 = fma(si, P.inv, fma(-half, P.m, half));
    const double lo_clamp = -(double)kPad, hi_clamp = (double)(N + kPad - 2);
    T acc = T(0);

    if (P.axis) {
        // The ray stays in one column (or row) of pixels; on a pixel edge it is split
        // evenly between the two pixels that share the edge.
        const double uc = fmin(fmax(u0, lo_clamp), hi_clamp);
        const double nearest = rint(uc);
        int c0;
        T w0, w1;
        if (fabs(uc - nearest) <= kEdgeTie) {
            c0 = (int)nearest - 1;
            w0 = w1 = T(0.5 * P.len);
        } else {
            c0 = (int)floor(uc);
            w0 = T(P.len);
            w1 = T(0);
        }
        if (u0 < lo_clamp || u0 > hi_clamp) c0 = -kPad;   // outside: read zero padding
        c0 = min(max(c0, -kPad), N + kPad - 2);           // both taps inside the padded row
        const T *p = img + c0;
        for (int r = 0; r < N; ++r) {
            acc = fma(w0, p[0], acc);
            acc = fma(w1, p[1], acc);
            p += S;
        }
    } else {
        // Band r holds the minor-axis interval [lo_r, lo_r + |m|], lo_r = lo0 + r*m.
        const double lo0 = u0 + fmin(P.m, 0.0);
        const double am = fabs(P.m);
        double ra, rb;
        if (P.m > 0.0) {
            ra = (-1.0 - am - lo0) / am;
            rb = (N + 1.0 - lo0) / am;
        } else {
            ra = (lo0 - (N + 1.0)) / am;
            rb = (lo0 + 1.0 + am) / am;
        }
        ra = fmin(fmax(ra, 0.0), (double)N);
        rb = fmin(fmax(rb, 0.0), (double)N);
        int r0 = (int)floor(ra);
        int r1 = min((int)ceil(rb) + 1, N);
        if (i >= n_det) {
            r0 = N;
            r1 = 0;
        }
        // wave-uniform band range: lanes outside their own chord read zero padding
        const int wr0 = __builtin_amdgcn_readfirstlane(wave_min_i(r0));
        const int wr1 = __builtin_amdgcn_readfirstlane(wave_max_i(r1));
        Band<T> band(fma((double)wr0, P.m, lo0), P.m);
        // row-start pointer (padding included): column offsets are unsigned
        const T *row = img - kPad + (size_t)wr0 * S;
        const BandWeights<T> bw(P.invq, P.len);
        const unsigned cmax = (unsigned)(N + 2 * kPad - 2);
        int r = wr0;
        // four bands per trip, all loads issued before their use
        for (; r + 4 <= wr1; r += 4) {
            unsigned c[4];
            T w[4], v0[4], v1[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                c[j] = band.column(cmax);
                w[j] = band.left_length(bw);
                band.next();
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const Taps<T> t = load_taps(row + (size_t)j * S, c[j]);
                v0[j] = t.a;
                v1[j] = t.b;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                acc = fma(w[j], v0[j], acc);
                acc = fma(bw.len - w[j], v1[j], acc);
            }
            row += 4 * (size_t)S;
        }
        for (; r < wr1; ++r) {
            const unsigned c = band.column(cmax);
            const T w = band.left_length(bw);
            band.next();
            const Taps<T> t = load_taps(row, c);
            acc = fma(w, t.a, acc);
            acc = fma(bw.len - w, t.b, acc);
            row += S;
        }
    }
    if (i < n_det) y[(size_t)a * n_det + i] = acc;
}

}  // namespace
}  // namespace abg
