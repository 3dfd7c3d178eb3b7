// Device code of the ray-driven forward projector (line model), shared by the
// single-problem kernels (projectors.hip) and the batched kernels (batch.hip), so that
// both run the same arithmetic.
#pragma once

#include <cmath>

#include "abg_internal.h"
#include "footprint.h"

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
    // lo: the band's lower minor-axis edge in padded column coordinates (+ kPad), so that
    // floor(lo) is the padded column itself
    double lo, m;
    __device__ Band(double lo0, double m_) : lo(lo0 + kPad), m(m_) {}
    __device__ void next() { lo += m; }
    __device__ unsigned column(unsigned cmax) const
    {
        return min((unsigned)(int)floor(lo), cmax);
    }
    // padded column, unclamped, by truncation. A wave walks only the bands some lane's
    // ray crosses (at most N of them, |m| <= 1), and the lanes of a wave lie within 63
    // bins of each other (63 * 64 * sqrt(2) < 5702 px for the spacings a geometry
    // accepts), so every column a walking lane reaches is below 2N + 5710 < 2^17 in
    // magnitude (N <= 32768): the conversion is exact and the byte offset cannot wrap back
    // into the row. A tap can meet a nonzero pixel only for lo >= kPad - 1 > 0, where
    // truncation is floor; below, truncation lands in the zero padding (lo > -1) or before
    // the row (out of range, read as zero) as floor would.
    __device__ int column_raw() const { return (int)lo; }
    // length of the band segment left of the pixel edge at floor(lo) + 1, from the
    // fractional part of lo (exactly lo - floor(lo) for lo >= 0)
    __device__ double left_length(const BandWeights<double> &b) const
    {
        const double t = fma(-__builtin_amdgcn_fract(lo), b.invq, b.invq);
        // min of two finite values: the plain instruction (fmin would quieten the
        // loop-invariant operand on every step); the length is the same in every lane
        // (a wave walks one angle), so a scalar operand holds it
        double w;
        asm("v_min_f64 %0, %1, %2" : "=v"(w) : "s"(b.len), "v"(t));
        return w;
    }
    // (lo - floor(lo)) * s
    __device__ double frac_scaled(double s) const { return (lo - floor(lo)) * s; }
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
    __device__ int column_raw() const { return c; }
    __device__ float left_length(const BandWeights<float> &b) const
    {
        const float w = fmaf((float)f, -b.invq * 0x1p-32f, b.invq);
        return __builtin_amdgcn_fmed3f(w, b.len, -1e30f);   // min(w, len)
    }
    // fractional part times s * 2^32 (the caller folds 2^-32 into s)
    __device__ float frac_scaled(float s) const { return (float)f * s; }
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

// The same two taps through a buffer resource spanning exactly one padded row of S
// elements: the hardware range check returns zero for a column outside the row (a lane
// walking bands outside its own chord, negative columns included, as their unsigned byte
// offset is huge), so the walk needs no clamp.
template <typename T>
__device__ inline Taps<T> load_taps_row(const T *row, int S, int col)
{
    __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<T *>(row), (short)0, S * (int)sizeof(T), kRawBufferFlags);
    const int boff = col * (int)sizeof(T);
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(Taps<T>, __builtin_amdgcn_raw_buffer_load_b64(r, boff, 0, 0));
    } else {
        return __builtin_bit_cast(Taps<T>, __builtin_amdgcn_raw_buffer_load_b128(r, boff, 0, 0));
    }
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
        // row-start pointer (padding included); taps outside the padded row read zero
        const T *row = img - kPad + (size_t)wr0 * S;
        const BandWeights<T> bw(P.invq, P.len);
        int r = wr0;
        // kTrip bands per trip, their loads issued before their use. Two is the measured
        // best on gfx950 (FP64 at 2048^2: 15% below four; one and three are slower, FP32
        // is flat): a deeper trip holds more registers in flight without more memory
        // parallelism, since eight resident waves per SIMD already cover the gather
        // latency.
        constexpr int kTrip = 2;
        for (; r + kTrip <= wr1; r += kTrip) {
            int c[kTrip];
            T w[kTrip], v0[kTrip], v1[kTrip];
#pragma unroll
            for (int j = 0; j < kTrip; ++j) {
                c[j] = band.column_raw();
                w[j] = band.left_length(bw);
                band.next();
            }
#pragma unroll
            for (int j = 0; j < kTrip; ++j) {
                const Taps<T> t = load_taps_row(row + (size_t)j * S, S, c[j]);
                v0[j] = t.a;
                v1[j] = t.b;
            }
#pragma unroll
            for (int j = 0; j < kTrip; ++j) {
                acc = fma(w[j], v0[j], acc);
                acc = fma(bw.len - w[j], v1[j], acc);
            }
            row += kTrip * (size_t)S;
        }
        for (; r < wr1; ++r) {
            const int c = band.column_raw();
            const T w = band.left_length(bw);
            band.next();
            const Taps<T> t = load_taps_row(row, S, c);
            acc = fma(w, t.a, acc);
            acc = fma(bw.len - w, t.b, acc);
            row += S;
        }
    }
    if (i < n_det) y[(size_t)a * n_det + i] = acc;
}

// ---- strip and interpolation (Joseph) models -----------------------------------------
// Both walk the bands of the line model. Joseph samples each band on its centre line:
// the ray crosses it at minor coordinate u* = u0 + (r + 1/2) m, and with b = u* - 1/2
// (pixel-centre coordinates) the pixels floor(b) and floor(b) + 1 get (1 - frac b)/p and
// (frac b)/p. The strip model (a strip of width ds around the ray; area of strip and
// pixel over ds) weighs every pixel of the band whose centre lies within R pixels of b,
// R = ((p + q)/2 + ds/2)/p, by the line-model trapezoid integrated over the strip: with
// e = |b - c| p the centre's distance from the ray in detector units,
//     w = (G(e + ds/2) - G(e - ds/2)) / ds,   G = antiderivative of the trapezoid.
// For ds <= 1.4 that is at most four consecutive pixels, fetched with one 16-byte load.

// Bands [r0, r1) whose minor-axis interval, widened by `extra` pixels on both sides, can
// meet [-1, N + 1]; empty for rays that store nothing.
__device__ inline void band_range(double lo0, double m, int N, double extra, bool live, int &r0,
                                  int &r1)
{
    const double am = fabs(m);
    double ra, rb;
    if (m > 0.0) {
        ra = (-1.0 - am - extra - lo0) / am;
        rb = (N + 1.0 + extra - lo0) / am;
    } else {
        ra = (lo0 - extra - (N + 1.0)) / am;
        rb = (lo0 + 1.0 + am + extra) / am;
    }
    ra = fmin(fmax(ra, 0.0), (double)N);
    rb = fmin(fmax(rb, 0.0), (double)N);
    r0 = live ? (int)floor(ra) : N;
    r1 = live ? min((int)ceil(rb) + 1, N) : 0;
}

template <typename T> struct alignas(sizeof(T)) Quad {
    T v[4];
};

// Joseph's model, ray i of angle a (called by whole waves of consecutive rays).
template <typename T>
__device__ inline void forward_ray_joseph(const T *__restrict__ xr, const T *__restrict__ xc,
                                          T *__restrict__ y, const AngleParams *__restrict__ ang,
                                          int a, int i, int N, int S, int n_det, double ds,
                                          double s0)
{
    const AngleParams P = ang[a];
    const T *img = (P.steep ? xr : xc) + kPad;
    const double half = 0.5 * N;
    const double si = s0 + (double)i * ds;
    const double u0 = fma(si, P.inv, fma(-half, P.m, half));
    T acc = T(0);
    if (P.axis) {
        // u* is the same in every band; out of reach, both taps read zero padding
        const double b = fmin(fmax(u0 - 0.5, -(double)kPad), (double)(N + kPad - 2));
        const int c0 = (int)floor(b);
        const T w1 = T((b - c0) * P.len), w0 = T(P.len) - w1;
        const T *p = img + c0;
        for (int r = 0; r < N; ++r) {
            acc = fma(w0, p[0], acc);
            acc = fma(w1, p[1], acc);
            p += S;
        }
    } else {
        const double lo0 = u0 + fmin(P.m, 0.0);
        int r0, r1;
        band_range(lo0, P.m, N, 0.0, i < n_det, r0, r1);
        const int wr0 = __builtin_amdgcn_readfirstlane(wave_min_i(r0));
        const int wr1 = __builtin_amdgcn_readfirstlane(wave_max_i(r1));
        // b at band wr0
        Band<T> band(fma((double)wr0 + 0.5, P.m, u0) - 0.5, P.m);
        const T *row = img - kPad + (size_t)wr0 * S;
        const T len = T(P.len);
        const T fs = sizeof(T) == 4 ? T(P.len * 0x1p-32) : len;
        const unsigned cmax = (unsigned)(N + 2 * kPad - 2);
        int r = wr0;
        for (; r + 4 <= wr1; r += 4) {
            unsigned c[4];
            T w[4], v0[4], v1[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                c[j] = band.column(cmax);
                w[j] = band.frac_scaled(fs);
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
                acc = fma(len - w[j], v0[j], acc);
                acc = fma(w[j], v1[j], acc);
            }
            row += 4 * (size_t)S;
        }
        for (; r < wr1; ++r) {
            const unsigned c = band.column(cmax);
            const T w = band.frac_scaled(fs);
            band.next();
            const Taps<T> t = load_taps(row, c);
            acc = fma(len - w, t.a, acc);
            acc = fma(w, t.b, acc);
            row += S;
        }
    }
    if (i < n_det) y[(size_t)a * n_det + i] = acc;
}

// Strip model, ray i of angle a (called by whole waves of consecutive rays; ds <= 1.4).
template <typename T>
__device__ inline void forward_ray_strip(const T *__restrict__ xr, const T *__restrict__ xc,
                                         T *__restrict__ y, const AngleParams *__restrict__ ang,
                                         int a, int i, int N, int S, int n_det, double ds,
                                         double s0)
{
    const AngleParams P = ang[a];
    const T *img = P.steep ? xr : xc;   // row starts, padding included
    const double half = 0.5 * N;
    const double si = s0 + (double)i * ds;
    const double u0 = fma(si, P.inv, fma(-half, P.m, half));
    const double R = (P.half + 0.5 * ds) * P.len;     // reach in pixels
    const Trapezoid<T> tz(P, ds);
    const T pT = T(P.p);
    // pixel c0 + k of a band, with c0 = floor(b - R) + 1 and f = frac(b - R + 1), lies
    // b - c0 - k = f + (R - 1 - k) from the crossing point
    const T d0 = T(R - 1.0);
    const unsigned cmax = (unsigned)(S - 4);           // the four pixels stay in the row
    T acc = T(0);
    auto band4 = [&](T f, const Quad<T> &v) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const T e = fabs(f + (d0 - T(k))) * pT;
            acc = fma(tz.strip(e), v.v[k], acc);
        }
    };
    if (P.axis) {
        // first pixel (padded index) and f, clamped into the row: out of reach only
        // padding is read
        const double pb = fmin(fmax(u0 - 0.5 - R + 1.0 + kPad, 0.0), (double)(N + 2 * kPad - 4));
        const int c0 = (int)floor(pb);
        const T f = T(pb - c0);
        const T *p = img + c0;
        for (int r = 0; r < N; ++r) {
            const Quad<T> v = *reinterpret_cast<const Quad<T> *>(p);
            band4(f, v);
            p += S;
        }
    } else {
        const double lo0 = u0 + fmin(P.m, 0.0);
        int r0, r1;
        band_range(lo0, P.m, N, R, i < n_det, r0, r1);
        const int wr0 = __builtin_amdgcn_readfirstlane(wave_min_i(r0));
        const int wr1 = __builtin_amdgcn_readfirstlane(wave_max_i(r1));
        // b - R + 1 at band wr0
        Band<T> band(fma((double)wr0 + 0.5, P.m, u0) - 0.5 - R + 1.0, P.m);
        const T *row = img + (size_t)wr0 * S;
        const T fs = sizeof(T) == 4 ? T(0x1p-32) : T(1);
        int r = wr0;
        for (; r + 2 <= wr1; r += 2) {
            unsigned c[2];
            T f[2];
            Quad<T> v[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                c[j] = band.column(cmax);
                f[j] = band.frac_scaled(fs);
                band.next();
            }
#pragma unroll
            for (int j = 0; j < 2; ++j)
                v[j] = *reinterpret_cast<const Quad<T> *>(reinterpret_cast<const char *>(
                    row + (size_t)j * S) + c[j] * (unsigned)sizeof(T));
#pragma unroll
            for (int j = 0; j < 2; ++j) band4(f[j], v[j]);
            row += 2 * (size_t)S;
        }
        if (r < wr1) {
            const unsigned c = band.column(cmax);
            const T f = band.frac_scaled(fs);
            const Quad<T> v = *reinterpret_cast<const Quad<T> *>(
                reinterpret_cast<const char *>(row) + c * (unsigned)sizeof(T));
            band4(f, v);
        }
    }
    if (i < n_det) y[(size_t)a * n_det + i] = acc;
}

// ---- line model, four angles per block, band rows staged in LDS -------------------------
// The forward walk above issues one 64-lane gather per band and wave, and the texture
// path takes them at four lane addresses per cycle: that rate bounds it. A block of four
// adjacent angles (one wave each) and the same 64 rays reads nearly the same columns of
// every band row in all four waves, so here each band row's columns the block can touch
// are copied once into LDS by one 16-byte load per lane (a quarter of the addresses), and
// the waves read their taps from there. Everything else is the walk above, band by band
// in the same order: the results are the same bits. The LDS returns a band's taps no
// faster than the texture path does, so this walk alone is slower; run beside the
// direct walk in the same launch it takes its taps through the other unit.
//
// The window of band r starts at org(r) and holds kStageCols columns. For angle i the
// leftmost lane sits at lmin_i + r m_i and the rightmost at rmax_i + r m_i (padded
// columns; lanes are monotone in their offset), so the columns the block touches lie in
// [min_i(lmin_i + r m_i), max_i(rmax_i + r m_i) + 2]. The lower edge is concave in r and
// the upper convex, so their chords over the block's bands bound them from below and
// from above, and the window's width is checked at the two end bands only. org(r)
// follows the lower chord in 32.32 fixed point on the scalar unit. Blocks whose angles
// differ in orientation, include an axis-aligned or a missing angle, or need a wider
// window take the walk above.
constexpr int kStageBands = 8;
template <typename T> constexpr int kStageCols = 64 * 16 / (int)sizeof(T);

template <typename T> struct FwdStageLds {
    T win[2][kStageBands][kStageCols<T>];
    double lmin[4], rmax[4], m[4];
    int r0[4], r1[4], kind[4];
};

__device__ inline double lane_value_f64(double v, int l)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, l);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ inline long long uniform_ll(long long v)
{
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

// Angles a0 .. a0 + 3 (wave w takes a0 + w), rays ray0 .. ray0 + 63 of each. All four
// waves call it (also for angles past n_ang); it starts with a block-wide barrier, so
// that consecutive calls of a block may share L.
template <typename T>
__device__ inline void forward_block_staged(const T *__restrict__ xr, const T *__restrict__ xc,
                                            T *__restrict__ y, const AngleParams *__restrict__ ang,
                                            int a0, int ray0, int N, int S, int n_ang, int n_det,
                                            double ds, double s0, FwdStageLds<T> &L)
{
    constexpr int W = kStageCols<T>;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int a = a0 + wave, i = ray0 + lane;
    int kind = 0, wr0 = 0, wr1 = 0;
    double lo0 = 0.0, lmin = 0.0, rmax = 0.0, m = 0.0;
    AngleParams P{};
    if (a < n_ang) {
        P = ang[a];
        if (!P.axis) {
            kind = P.steep ? 1 : 2;
            const double half = 0.5 * N;
            const double si = s0 + (double)i * ds;
            const double u0 = fma(si, P.inv, fma(-half, P.m, half));
            lo0 = u0 + fmin(P.m, 0.0);
            int r0, r1;
            band_range(lo0, P.m, N, 0.0, i < n_det, r0, r1);
            wr0 = __builtin_amdgcn_readfirstlane(wave_min_i(r0));
            wr1 = __builtin_amdgcn_readfirstlane(wave_max_i(r1));
            const double l0 = lane_value_f64(lo0, 0), l63 = lane_value_f64(lo0, 63);
            lmin = fmin(l0, l63) + kPad;
            rmax = fmax(l0, l63) + kPad;
            m = P.m;
        }
    }
    __syncthreads();                                   // the previous call is done with L
    if (lane == 0) {
        L.kind[wave] = kind;
        L.r0[wave] = wr0;
        L.r1[wave] = wr1;
        L.lmin[wave] = lmin;
        L.rmax[wave] = rmax;
        L.m[wave] = m;
    }
    __syncthreads();
    // the block's choice, the same in every wave
    bool staged = L.kind[0] != 0;
    int rb0 = N, rb1 = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        staged = staged && L.kind[v] == L.kind[0];
        rb0 = min(rb0, L.r0[v]);
        rb1 = max(rb1, L.r1[v]);
    }
    double lb = 1e300, le = 1e300, hb = -1e300, he = -1e300;
    if (staged && rb0 < rb1) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            lb = fmin(lb, fma((double)rb0, L.m[v], L.lmin[v]));
            le = fmin(le, fma((double)(rb1 - 1), L.m[v], L.lmin[v]));
            hb = fmax(hb, fma((double)rb0, L.m[v], L.rmax[v]));
            he = fmax(he, fma((double)(rb1 - 1), L.m[v], L.rmax[v]));
        }
        // taps reach 2 columns right of a lane's position (truncation of a negative
        // position adds one); org sits 2 below the lower chord
        staged = fmax(hb - lb, he - le) + 6.0 <= (double)W;
    }
    if (!staged) {
        if (a < n_ang) forward_ray(xr, xc, y, ang, a, i, N, S, n_det, ds, s0);
        return;
    }
    T acc = T(0);
    if (rb0 < rb1) {
        const T *img = L.kind[0] == 1 ? xr : xc;       // padded rows
        const double slope = rb1 - 1 > rb0 ? (le - lb) / (double)(rb1 - 1 - rb0) : 0.0;
        const long long ofx0 = uniform_ll(__double2ll_rn((lb - 2.0) * 0x1p32));
        const long long dfx = uniform_ll(__double2ll_rn(slope * 0x1p32));
        auto org_of = [&](int r) { return (int)((ofx0 + (long long)(r - rb0) * dfx) >> 32); };
        auto stage = [&](int cb, int par) {
#pragma unroll
            for (int q = 0; q < kStageBands / 4; ++q) {
                const int r = cb + wave + 4 * q;
                if (r < rb1) {
                    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                        const_cast<T *>(img + (size_t)r * S), (short)0, S * (int)sizeof(T),
                        kRawBufferFlags);
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(
                        rs, (__attribute__((address_space(3))) void *)&L.win[par][r - cb][0], 16,
                        org_of(r) * (int)sizeof(T) + lane * 16, 0, 0, 0);
                }
            }
        };
        Band<T> band(fma((double)wr0, P.m, lo0), P.m);
        const BandWeights<T> bw(P.invq, P.len);
        stage(rb0, 0);
        int par = 0;
        for (int cb = rb0; cb < rb1; cb += kStageBands, par ^= 1) {
            __builtin_amdgcn_s_waitcnt(0);                 // this wave's rows have landed
            __syncthreads();                               // every wave's rows, and the other
                                                           // buffer is free again
            if (cb + kStageBands < rb1) stage(cb + kStageBands, par ^ 1);
            const int e0 = max(cb, wr0), e1 = min(cb + kStageBands, wr1);
            for (int r = e0; r < e1; ++r) {
                const int c = band.column_raw();
                const T w = band.left_length(bw);
                band.next();
                // the column within the window as one vector value (kept whole, so that
                // both taps come from one address)
                int off = c - org_of(r);
                asm volatile("" : "+v"(off));
                const Taps<T> t = *reinterpret_cast<const Taps<T> *>(&L.win[par][r - cb][off]);
                acc = fma(w, t.a, acc);
                acc = fma(bw.len - w, t.b, acc);
            }
        }
    }
    if (a < n_ang && i < n_det) y[(size_t)a * n_det + i] = acc;
}

}  // namespace
}  // namespace abg
