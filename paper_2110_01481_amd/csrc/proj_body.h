// Device code of the projectors, shared by the single-problem kernels (projectors.hip)
// and the batched kernels (batch.hip), so that both run the same arithmetic.
#pragma once

#include <cmath>

#include "abg_internal.h"

namespace abg {
namespace {


constexpr int kFwdBlock = 256;
// An axis-aligned ray lies on a pixel edge when its offset from the edge is below this
// (in pixels): bin positions carry rounding error, and an edge ray in exact arithmetic
// must split evenly. FP32 back projection evaluates offsets with ~4e-6 error.
constexpr double kEdgeTie = 1e-9;
template <typename T> __device__ inline T edge_tie();
template <> __device__ inline double edge_tie<double>() { return 1e-9; }
template <> __device__ inline float edge_tie<float>() { return 2e-5f; }
// back projector: a 16 x 16 pixel tile per block, 4 pixels per lane, the 8 waves
// splitting the angles; the tile's detector footprint for a block of angles (64 or 128) is staged per
// round (at most 30 bins per angle for det_spacing >= 0.75, plus margins)
constexpr int kTile = 16;
constexpr int kBackWaves = 8;
constexpr int kBackThreads = 64 * kBackWaves;
constexpr int kPixPerLane = kTile * kTile / 64;
constexpr int kAngBlock = 128;
constexpr int kWin = 32;

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

// Per staged angle: position of the tile's reference pixel in the window (f), the
// change of u per pixel step (cu, su), the window's first bin, and the line-model
// trapezoid of the matched back projector.
template <typename T>
struct alignas(16) BackStage {
    T f, cu, su, su4;   // su4 = 4 su, the step between a lane's pixel rows
    T invp, half, invpq;
    int axis;
};

// Length of a ray at offset |t| from a unit pixel's centre projection (the trapezoid of
// the line model); on an axis-aligned ray at exactly |t| = 1/2 the two pixels share it.
template <typename T>
__device__ inline T trapezoid(T at, const BackStage<T> &P)
{
    if (P.axis) {
        if (fabs(at - T(0.5)) <= edge_tie<T>()) return T(0.5) * P.invp;
        return at < T(0.5) ? P.invp : T(0);
    }
    return fmin(P.invp, fmax(T(0), (P.half - at) * P.invpq));
}

template <typename T> __device__ inline T fract_of(T u);
template <> __device__ inline float fract_of<float>(float u) { return __builtin_amdgcn_fractf(u); }
template <> __device__ inline double fract_of<double>(double u) { return __builtin_amdgcn_fract(u); }

// Staged window entry: the bin's value and the difference to the next bin.
template <typename T> struct alignas(2 * sizeof(T)) BinPair {
    T v, d;
};

// One pixel's contribution at detector coordinate u (window-relative). The window starts
// at least one bin below the tile's smallest u, and a 16 x 16 tile spans at most
// 15 sqrt(2) / ds < 28.3 bins for ds >= 0.75 (the smallest spacing a geometry accepts),
// so 1 <= u < 30.3 up to rounding: truncation is floor and k <= kWin - 2.
template <typename T, bool ADJ>
__device__ inline T back_tap(const BinPair<T> *wrow, T u, const BackStage<T> &P, T dsT)
{
    const T w = fract_of(u);
    const int k = (int)u;
    const BinPair<T> b = wrow[k];
    if (!ADJ) return fma(w, b.d, b.v);
    return trapezoid(w * dsT, P) * b.v + trapezoid((T(1) - w) * dsT, P) * (b.v + b.d);
}

// LDS of one back-projection block (declared by the calling kernel, so that a kernel
// serving both back projectors holds one copy). AB angles are staged per round; the
// per-angle set-up is double-buffered (round r is computed while round r + 1's is
// written); the waves' partial sums reuse the window's space at the end of a tile.
template <typename T, int AB = kAngBlock> struct BackLds {
    union {
        BinPair<T> win[AB][kWin];
        T part[kBackWaves - 1][kTile * kTile];
    };
    BackStage<T> prm[2][AB];
    int ib[2][AB];      // first bin of each angle's window
};

// The 16 x 16 tile with first column c0 and first row r0, by one block of kBackThreads.
// Starts and ends with a block-wide barrier, so consecutive calls may share the LDS.
//
// Software pipeline over rounds of AB angles: the sinogram loads of round r + 1's windows
// are issued before round r is computed and land in LDS after it, and the angle
// parameters are fetched one round before their set-up, so neither waits on the memory
// latency in the barrier-separated phases. The loads are branch-free (clamped addresses,
// out-of-range bins zeroed when stored).
//
// PAD: instead of x, the tile goes to the forward projector's zero-padded row-major and
// transposed copies xr, xc (row stride S, image column c at c + kPad; the padding must
// already be zero), through LDS so that both writes are coalesced.
template <typename T, bool ADJ, int AB = kAngBlock, bool PAD = false>
__device__ inline void back_tile(const T *__restrict__ y, T *__restrict__ x,
                                 const AngleParams *__restrict__ ang, int N, int n_ang,
                                 int n_det, double ds, double s0, int c0, int r0,
                                 BackLds<T, AB> &L, T *__restrict__ xr = nullptr,
                                 T *__restrict__ xc = nullptr, int S = 0)
{
    static_assert(AB <= kBackThreads, "one thread sets up one angle");
    constexpr int kIt = AB * kWin / kBackThreads;      // window entries per thread and round
    constexpr int kRowsPer = kBackThreads / kWin;      // angles covered by one pass
    static_assert(kIt * kBackThreads == AB * kWin && 2 * kIt <= 32, "window split");
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // lane owns pixels (tx, ty0 + 4j), j = 0..3, of the 16 x 16 tile
    const int tx = lane & 15, ty0 = lane >> 4;
    const double xref = c0 - 0.5 * N + 0.5, yref = r0 - 0.5 * N + 0.5;
    const double s0u = s0 / ds;
    const T ftx = T(tx), fty = T(ty0);
    const T dsT = T(ds);
    const int n_rounds = (n_ang + AB - 1) / AB;
    const int kk = threadIdx.x % kWin;                 // this thread's window column

    AngleParams Pn;                                    // parameters of the next set-up
    auto fetch = [&](int r) { Pn = ang[min(r * AB + (int)threadIdx.x, n_ang - 1)]; };
    auto setup = [&](int r) {
        if ((int)threadIdx.x < min(AB, n_ang - r * AB)) {
            const double uref = fma(xref, Pn.cu, fma(yref, Pn.su, -s0u));
            const double umin = uref + (kTile - 1) * (fmin(Pn.cu, 0.0) + fmin(Pn.su, 0.0));
            const double ib = floor(umin) - 1.0;
            BackStage<T> st;
            st.f = T(uref - ib);
            st.cu = T(Pn.cu);
            st.su = T(Pn.su);
            st.su4 = T(4.0 * Pn.su);
            st.invp = T(Pn.len);
            st.half = T(Pn.half);
            st.invpq = T(Pn.invpq);
            st.axis = Pn.axis;
            L.prm[r & 1][threadIdx.x] = st;
            L.ib[r & 1][threadIdx.x] = (int)ib;
        }
    };
    T w0[kIt], w1[kIt];
    unsigned live = 0;                                 // in-range bits of w0 / w1
    auto load = [&](int r) {
        const int a0 = r * AB, last = min(AB, n_ang - a0) - 1;
        live = 0;
#pragma unroll
        for (int j = 0; j < kIt; ++j) {
            const int t = min((int)threadIdx.x / kWin + j * kRowsPer, last);
            const int bin = L.ib[r & 1][t] + kk;
            const T *row = y + (size_t)(a0 + t) * n_det;
            w0[j] = row[min(max(bin, 0), n_det - 1)];
            w1[j] = row[min(max(bin + 1, 0), n_det - 1)];
            live |= (unsigned)(bin >= 0 && bin < n_det) << (2 * j);
            live |= (unsigned)(bin + 1 >= 0 && bin + 1 < n_det) << (2 * j + 1);
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int j = 0; j < kIt; ++j) {
            const T v0 = (live >> (2 * j)) & 1u ? w0[j] : T(0);
            const T v1 = (live >> (2 * j + 1)) & 1u ? w1[j] : T(0);
            L.win[(int)threadIdx.x / kWin + j * kRowsPer][kk] = BinPair<T>{v0, v1 - v0};
        }
    };

    T acc[kPixPerLane] = {};
    __syncthreads();                                   // the previous tile is done with the LDS
    fetch(0);
    setup(0);
    if (n_rounds > 1) fetch(1);
    __syncthreads();
    load(0);
    for (int r = 0; r < n_rounds; ++r) {
        const int na = min(AB, n_ang - r * AB);
        __syncthreads();                               // round r - 1 is done with win, prm
        store();
        if (r + 1 < n_rounds) {
            setup(r + 1);
            if (r + 2 < n_rounds) fetch(r + 2);
        }
        __syncthreads();                               // window r, set-up r + 1 visible
        if (r + 1 < n_rounds) load(r + 1);
        // the block's waves take interleaved angles of the round
        for (int t = wave; t < na; t += kBackWaves) {
            const BackStage<T> P = L.prm[r & 1][t];
            const T u0 = fma(ftx, P.cu, fma(fty, P.su, P.f));
            acc[0] += back_tap<T, ADJ>(L.win[t], u0, P, dsT);
#pragma unroll
            for (int j = 1; j < kPixPerLane; ++j)
                acc[j] += back_tap<T, ADJ>(L.win[t], fma(T(j), P.su4, u0), P, dsT);
        }
    }
    // fixed-order sum of the waves' partials
    __syncthreads();                                   // the window space becomes part
#pragma unroll
    for (int j = 0; j < kPixPerLane; ++j) {
        const int pix = (ty0 + 4 * j) * kTile + tx;
        if (wave > 0) L.part[wave - 1][pix] = acc[j];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int j = 0; j < kPixPerLane; ++j) {
            const int pix = (ty0 + 4 * j) * kTile + tx;
            T sum = acc[j];
#pragma unroll
            for (int v = 0; v < kBackWaves - 1; ++v) sum += L.part[v][pix];
            const T val = ADJ ? sum : sum * T(1.0 / ds);
            const int c = c0 + tx, r = r0 + ty0 + 4 * j;
            if constexpr (PAD) L.part[0][pix] = val;   // the lane's own entry
            else if (r < N && c < N) x[(size_t)r * N + c] = val;
        }
    }
    if constexpr (PAD) {
        static_assert(kBackThreads >= kTile * kTile, "one thread per pixel of the tile");
        __syncthreads();
        const int t = threadIdx.x, hi = t / kTile, lo = t % kTile;
        // xr: 16 lanes write 16 consecutive columns of a row; xc: of a column
        if (t < kTile * kTile) {
            if (r0 + hi < N && c0 + lo < N) xr[(size_t)(r0 + hi) * S + kPad + c0 + lo] = L.part[0][hi * kTile + lo];
            if (c0 + hi < N && r0 + lo < N) xc[(size_t)(c0 + hi) * S + kPad + r0 + lo] = L.part[0][lo * kTile + hi];
        }
    }
    __syncthreads();
}

}  // namespace
}  // namespace abg
