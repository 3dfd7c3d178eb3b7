// Device code of the pixel-driven back projectors (linear interpolation B, and the
// line-model transpose A^T), shared by the single-problem kernels (projectors.hip) and the
// batched kernels (batch.hip), so that both run the same arithmetic.
#pragma once

#include <cmath>

#include "abg_internal.h"
#include "footprint.h"

namespace abg {
namespace {

// An axis-aligned ray lies on a pixel edge when its offset from the edge is below this
// (in pixels); FP32 back projection evaluates offsets with ~4e-6 error.
template <typename T> __device__ inline T edge_tie();
template <> __device__ inline double edge_tie<double>() { return 1e-9; }
template <> __device__ inline float edge_tie<float>() { return 2e-5f; }

// back projector: a 16 x 16 pixel tile per block, 4 pixels per lane, the 8 waves
// splitting the angles; the tile's detector footprint for a block of angles (64 or 128)
// is staged per round (at most 30 bins per angle for det_spacing >= 0.75, plus margins)
constexpr int kTile = 16;
constexpr int kBackWaves = 8;
constexpr int kBackThreads = 64 * kBackWaves;
// Launch bound (waves per SIMD) of the back projector kernels: the interpolating kind in
// FP32 at most 64 VGPRs (four blocks, eight waves per SIMD, share a CU), in FP64 at most
// 80 (six waves); the matched kind's FP64 trapezoid needs more registers than that
// without spilling.
template <typename T, bool ADJ = false> constexpr int kBackMinWaves = ADJ ? 1 : 6;
template <> constexpr int kBackMinWaves<float, false> = 8;
template <> constexpr int kBackMinWaves<float, true> = 8;
constexpr int kPixPerLane = kTile * kTile / 64;
constexpr int kAngBlock = 128;
constexpr int kWin = 32;

// Per staged angle: position of the tile's reference pixel in the window (f), the
// change of u per pixel step (cu, su), the window's first bin, and the line-model
// trapezoid of the matched back projector.
template <typename T>
struct alignas(16) BackStage {
    T f, cu, su, su4;   // su4 = 4 su, the step between a lane's pixel rows
    // matched back projector: with w = frac(u), the trapezoid's values at the two bins
    // around u are clamp(t1 - w c, 0, 1/p) (distance w ds) and clamp(t2 + w c, 0, 1/p)
    // (distance (1 - w) ds), where t1 = h/(pq), t2 = (h - ds)/(pq), c = ds/(pq), h = (p+q)/2
    T invp, t1, t2, c;
    int axis;
};

// Length of an axis-aligned ray at offset |t| from a unit pixel's centre projection (the
// line model's trapezoid is then a box); at exactly |t| = 1/2 the two pixels share it.
template <typename T>
__device__ inline T box(T at, const BackStage<T> &P)
{
    if (fabs(at - T(0.5)) <= edge_tie<T>()) return T(0.5) * P.invp;
    return at < T(0.5) ? P.invp : T(0);
}

template <typename T> __device__ inline T clamp_to(T v, T hi);
template <> __device__ inline float clamp_to<float>(float v, float hi)
{
    return __builtin_amdgcn_fmed3f(v, 0.f, hi);
}
template <> __device__ inline double clamp_to<double>(double v, double hi)
{
    return fmin(hi, fmax(0.0, v));
}

template <typename T> __device__ inline T fract_of(T u);
template <> __device__ inline float fract_of<float>(float u) { return __builtin_amdgcn_fractf(u); }
template <> __device__ inline double fract_of<double>(double u) { return __builtin_amdgcn_fract(u); }

// One element at byte offset `off` of a raw buffer resource (zero past its size).
template <typename T> __device__ inline T buffer_elem(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

// Staged window entry: the bin's value and the difference to the next bin.
template <typename T> struct alignas(2 * sizeof(T)) BinPair {
    T v, d;
};

// One pixel's contribution at detector coordinate u (window-relative). The window starts
// at least one bin below the tile's smallest u, and a 16 x 16 tile spans at most
// 15 sqrt(2) / ds < 28.3 bins for ds >= 0.75 (the smallest spacing a geometry accepts),
// so 1 <= u < 30.3 up to rounding: truncation is floor and k <= kWin - 2.
// Adds the pixel's contribution to acc.
template <typename T, bool ADJ>
__device__ inline void back_tap(T &acc, const BinPair<T> *wrow, T u, const BackStage<T> &P, T dsT)
{
    const T w = fract_of(u);
    const int k = (int)u;
    const BinPair<T> b = wrow[k];
    if (!ADJ) {
        acc += fma(w, b.d, b.v);
        return;
    }
    T a0, a1;
    if (P.axis) {
        a0 = box(w * dsT, P);
        a1 = box((T(1) - w) * dsT, P);
    } else {
        a0 = clamp_to(fma(-w, P.c, P.t1), P.invp);
        a1 = clamp_to(fma(w, P.c, P.t2), P.invp);
    }
    acc = fma(a0, b.v, acc);
    acc = fma(a1, b.v + b.d, acc);
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

// Fixed-order sum of the waves' partials of a tile (the window space of the LDS becomes
// `part`), scaled, into x or (PAD) into the forward projector's padded copies xr / xc;
// ends with a block-wide barrier.
template <typename T, bool PAD>
__device__ inline void tile_store(const T (&acc)[kPixPerLane], T (*part)[kTile * kTile], T scale,
                                  T *__restrict__ x, int N, int c0, int r0, T *__restrict__ xr,
                                  T *__restrict__ xc, int S)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tx = lane & 15, ty0 = lane >> 4;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPixPerLane; ++j) {
        const int pix = (ty0 + 4 * j) * kTile + tx;
        if (wave > 0) part[wave - 1][pix] = acc[j];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int j = 0; j < kPixPerLane; ++j) {
            const int pix = (ty0 + 4 * j) * kTile + tx;
            T sum = acc[j];
#pragma unroll
            for (int v = 0; v < kBackWaves - 1; ++v) sum += part[v][pix];
            const T val = sum * scale;
            const int c = c0 + tx, r = r0 + ty0 + 4 * j;
            if constexpr (PAD) part[0][pix] = val;   // the lane's own entry
            else if (r < N && c < N) x[(size_t)r * N + c] = val;
        }
    }
    if constexpr (PAD) {
        static_assert(kBackThreads >= kTile * kTile, "one thread per pixel of the tile");
        __syncthreads();
        const int t = threadIdx.x, hi = t / kTile, lo = t % kTile;
        // xr: 16 lanes write 16 consecutive columns of a row; xc: of a column
        if (t < kTile * kTile) {
            if (r0 + hi < N && c0 + lo < N) xr[(size_t)(r0 + hi) * S + kPad + c0 + lo] = part[0][hi * kTile + lo];
            if (c0 + hi < N && r0 + lo < N) xc[(size_t)(c0 + hi) * S + kPad + r0 + lo] = part[0][lo * kTile + hi];
        }
    }
    __syncthreads();
}

// The 16 x 16 tile with first column c0 and first row r0, by one block of kBackThreads.
// Starts and ends with a block-wide barrier, so consecutive calls may share the LDS.
//
// Software pipeline over rounds of AB angles: the sinogram loads of round r + 1's windows
// are issued before round r is computed and land in LDS after it, and the angle
// parameters are fetched one round before their set-up, so neither waits on the memory
// latency in the barrier-separated phases. The loads are branch-free (WY: out-of-range
// bins read as zero through the buffer's range check; otherwise clamped addresses, and
// out-of-range bins zeroed when stored).
//
// PAD: instead of x, the tile goes to the forward projector's zero-padded row-major and
// transposed copies xr, xc (row stride S, image column c at c + kPad; the padding must
// already be zero), through LDS so that both writes are coalesced.
//
// WY: the sinogram's bytes fit a 31-bit offset (the caller checks), so that the window
// loads go through one buffer resource over the whole sinogram (below); otherwise they
// clamp 64-bit addresses into the row.
template <typename T, bool ADJ, int AB = kAngBlock, bool PAD = false, bool WY = true>
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
    T ftx = T(tx), fty = T(ty0);
    const T dsT = T(ds);
    const int n_rounds = (n_ang + AB - 1) / AB;
    const int kk = threadIdx.x % kWin;                 // this thread's window column

    AngleParams Pn;                                    // parameters of the next set-up
    auto fetch = [&](int r) { Pn = ang[min(r * AB + (int)threadIdx.x, n_ang - 1)]; };
    auto setup = [&](int r) {
        if ((int)threadIdx.x < min(AB, n_ang - r * AB)) {
            // the tile's reference pixel and the first bin's offset, formed here from the
            // scalar arguments (opaque to hoisting: kept live across the rounds as FP64
            // vector registers, they would be spilled by the FP64 kernel at its six-wave
            // bound)
            int cx = c0, cy = r0;
            double s0v = s0;
            asm volatile("" : "+s"(cx), "+s"(cy), "+s"(s0v));
            const double xref = cx - 0.5 * N + 0.5, yref = cy - 0.5 * N + 0.5;
            const double s0u = s0v / ds;
            const double uref = fma(xref, Pn.cu, fma(yref, Pn.su, -s0u));
            const double umin = uref + (kTile - 1) * (fmin(Pn.cu, 0.0) + fmin(Pn.su, 0.0));
            const double ib = floor(umin) - 1.0;
            BackStage<T> st;
            st.f = T(uref - ib);
            st.cu = T(Pn.cu);
            st.su = T(Pn.su);
            st.su4 = T(4.0 * Pn.su);
            st.invp = T(Pn.len);
            st.t1 = T(Pn.half * Pn.invpq);
            st.t2 = T((Pn.half - ds) * Pn.invpq);
            st.c = T(ds * Pn.invpq);
            st.axis = Pn.axis;
            L.prm[r & 1][threadIdx.x] = st;
            L.ib[r & 1][threadIdx.x] = (int)ib;
        }
    };
    T w0[kIt], w1[kIt];
    unsigned live = 0;                                 // !WY: in-range bits of w0 / w1
    // WY: one buffer resource spans the sinogram (its bytes fit 31 bits), and the window
    // loads take 32-bit byte offsets instead of clamped 64-bit addresses. A bin outside
    // its detector row is read at offset 2^31, past the sinogram, which the range check
    // returns as zero: the loaded values need no mask. A bin inside its row has a
    // nonnegative element index below m, and 2^31 stays out of range if the compiler
    // moves a small constant between the offset and the instruction's offset field.
    const __amdgpu_buffer_rsrc_t ry = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<T *>(y), (short)0, WY ? (int)((size_t)n_ang * (size_t)n_det * sizeof(T)) : 0,
        kRawBufferFlags);
    constexpr unsigned kOutside = 0x80000000u;
    auto load = [&](int r) {
        const int a0 = r * AB, last = min(AB, n_ang - a0) - 1;
        live = 0;
        // WY: angles of the last round past n_ang are not clamped. Their window entries
        // are never read, and their loads, whatever first bin their stale (or never
        // written) LDS entries hold, go through the buffer's range check. Element index
        // of (angle a0 + t, bin 0), modulo 2^32:
        const unsigned row0 = (unsigned)(a0 + (int)threadIdx.x / kWin) * (unsigned)n_det;
#pragma unroll
        for (int j = 0; j < kIt; ++j) {
            const int t = (int)threadIdx.x / kWin + j * kRowsPer;
            if constexpr (WY) {
                // unsigned: a stale first bin must not overflow a signed sum
                const unsigned bin = (unsigned)L.ib[r & 1][t] + (unsigned)kk;
                const unsigned o = (row0 + (unsigned)(j * kRowsPer) * (unsigned)n_det + bin) *
                                   (unsigned)sizeof(T);
                w0[j] = buffer_elem<T>(ry, bin < (unsigned)n_det ? o : kOutside);
                w1[j] = buffer_elem<T>(ry, (bin + 1u < (unsigned)n_det ? o : kOutside) +
                                               (unsigned)sizeof(T));
            } else {
                const int tc = min(t, last);
                const int bin = L.ib[r & 1][tc] + kk;
                const T *row = y + (size_t)(a0 + tc) * n_det;
                w0[j] = row[min(max(bin, 0), n_det - 1)];
                w1[j] = row[min(max(bin + 1, 0), n_det - 1)];
                live |= (unsigned)((unsigned)bin < (unsigned)n_det) << (2 * j);
                live |= (unsigned)((unsigned)(bin + 1) < (unsigned)n_det) << (2 * j + 1);
            }
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int j = 0; j < kIt; ++j) {
            T v0 = w0[j], v1 = w1[j];
            if constexpr (!WY) {
                v0 = (live >> (2 * j)) & 1u ? v0 : T(0);
                v1 = (live >> (2 * j + 1)) & 1u ? v1 : T(0);
            }
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
            // FP64: keep the lane's pixel coordinates in registers (rematerialising them
            // costs two FP64 conversions per angle)
            if constexpr (sizeof(T) == 8) asm volatile("" : "+v"(ftx), "+v"(fty));
            const BackStage<T> P = L.prm[r & 1][t];
            const T u0 = fma(ftx, P.cu, fma(fty, P.su, P.f));
            if constexpr (!ADJ) {
                // the four window reads issued before their use
                BinPair<T> b[kPixPerLane];
                T w[kPixPerLane];
#pragma unroll
                for (int j = 0; j < kPixPerLane; ++j) {
                    const T u = j == 0 ? u0 : fma(T(j), P.su4, u0);
                    w[j] = fract_of(u);
                    b[j] = L.win[t][(int)u];
                }
#pragma unroll
                for (int j = 0; j < kPixPerLane; ++j) acc[j] += fma(w[j], b[j].d, b[j].v);
            } else {
                back_tap<T, ADJ>(acc[0], L.win[t], u0, P, dsT);
#pragma unroll
                for (int j = 1; j < kPixPerLane; ++j)
                    back_tap<T, ADJ>(acc[j], L.win[t], fma(T(j), P.su4, u0), P, dsT);
            }
        }
    }
    tile_store<T, PAD>(acc, L.part, ADJ ? T(1) : T(1.0 / ds), x, N, c0, r0, xr, xc, S);
}

// ---- transposes of the strip and interpolation (Joseph) models ------------------------
// Pixel driven like back_tile, over windows of plain sinogram values (kWinV bins per
// angle: a tile spans at most 28.3 bins for ds >= 0.75, plus two bins of margin on each
// side for the footprints). A pixel at window coordinate u (bins) takes the bins k with
// |k - u| below the footprint's reach, at most three:
//   Joseph^T:  (1/p) max(0, 1 - |k - u| ds / p)           (triangle of half-width p)
//   strip^T:   (G(e + ds/2) - G(e - ds/2)) / ds, e = |k - u| ds   (see Trapezoid)
constexpr int kWinV = 40;

template <typename T> struct alignas(16) BackStageV {
    T f, cu, su, su4;     // as BackStage
    T reach;              // footprint half-width in bins
    T js;                 // Joseph: ds / p^2;  strip: ds
    Trapezoid<T> tz;      // strip: footprint constants; Joseph: invp only
    T thr;                // B_tau: smallest entry kept
};

template <typename T, int AB = kAngBlock> struct BackLdsV {
    union {
        T win[AB][kWinV];
        T part[kBackWaves - 1][kTile * kTile];
    };
    BackStageV<T> prm[2][AB];
    int ib[2][AB];
};

// KIND ABG_BP_STRIP_TAU: the strip transpose without the entries below tau_thr (B_tau).
template <typename T, int KIND, int AB = kAngBlock, bool PAD = false>
__device__ inline void back_tile_v(const T *__restrict__ y, T *__restrict__ x,
                                   const AngleParams *__restrict__ ang, int N, int n_ang,
                                   int n_det, double ds, double s0, int c0, int r0,
                                   BackLdsV<T, AB> &L, T *__restrict__ xr = nullptr,
                                   T *__restrict__ xc = nullptr, int S = 0, double tau_thr = -1.0)
{
    static_assert(KIND == ABG_BP_STRIP_T || KIND == ABG_BP_JOSEPH_T || KIND == ABG_BP_STRIP_TAU,
                  "strip, Joseph or thresholded strip");
    static_assert(AB <= kBackThreads, "one thread sets up one angle");
    constexpr int kIt = AB * kWinV / kBackThreads;     // window entries per thread and round
    static_assert(kIt * kBackThreads == AB * kWinV && kIt <= 32, "window split");
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tx = lane & 15, ty0 = lane >> 4;
    const double xref = c0 - 0.5 * N + 0.5, yref = r0 - 0.5 * N + 0.5;
    const double s0u = s0 / ds;
    const T ftx = T(tx), fty = T(ty0);
    const int n_rounds = (n_ang + AB - 1) / AB;

    AngleParams Pn;
    auto fetch = [&](int r) { Pn = ang[min(r * AB + (int)threadIdx.x, n_ang - 1)]; };
    auto setup = [&](int r) {
        if ((int)threadIdx.x < min(AB, n_ang - r * AB)) {
            const double uref = fma(xref, Pn.cu, fma(yref, Pn.su, -s0u));
            const double umin = uref + (kTile - 1) * (fmin(Pn.cu, 0.0) + fmin(Pn.su, 0.0));
            const double ib = floor(umin) - 2.0;
            BackStageV<T> st;
            st.f = T(uref - ib);
            st.cu = T(Pn.cu);
            st.su = T(Pn.su);
            st.su4 = T(4.0 * Pn.su);
            st.tz = Trapezoid<T>(Pn, ds);
            st.thr = T(tau_thr);
            if (KIND == ABG_BP_JOSEPH_T) {
                st.reach = T(Pn.p / ds);
                st.js = T(ds * Pn.len * Pn.len);
            } else {
                st.reach = T((Pn.half + 0.5 * ds) / ds);
                st.js = T(ds);
            }
            L.prm[r & 1][threadIdx.x] = st;
            L.ib[r & 1][threadIdx.x] = (int)ib;
        }
    };
    T w0[kIt];
    unsigned live = 0;
    // entry e = threadIdx.x + j kBackThreads of a round is bin e % kWinV of angle e / kWinV
    auto load = [&](int r) {
        const int a0 = r * AB, last = min(AB, n_ang - a0) - 1;
        live = 0;
#pragma unroll
        for (int j = 0; j < kIt; ++j) {
            const int e = (int)threadIdx.x + j * kBackThreads;
            const int t = min(e / kWinV, last);
            const int bin = L.ib[r & 1][t] + e % kWinV;
            w0[j] = y[(size_t)(a0 + t) * n_det + min(max(bin, 0), n_det - 1)];
            live |= (unsigned)(bin >= 0 && bin < n_det) << j;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int j = 0; j < kIt; ++j) {
            const int e = (int)threadIdx.x + j * kBackThreads;
            L.win[e / kWinV][e % kWinV] = (live >> j) & 1u ? w0[j] : T(0);
        }
    };
    auto tap = [&](const T *win, T u, const BackStageV<T> &P) {
        // window coordinates keep u - reach >= 0.5, so truncation is floor
        const int k0 = (int)(u - P.reach) + 1;
        const T e0 = fabs(T(k0) - u), e1 = fabs(T(k0 + 1) - u), e2 = fabs(T(k0 + 2) - u);
        T w[3];
        if constexpr (KIND == ABG_BP_JOSEPH_T) {
            w[0] = fmax(fma(-e0, P.js, P.tz.invp), T(0));
            w[1] = fmax(fma(-e1, P.js, P.tz.invp), T(0));
            w[2] = fmax(fma(-e2, P.js, P.tz.invp), T(0));
        } else {
            w[0] = P.tz.strip(e0 * P.js);
            w[1] = P.tz.strip(e1 * P.js);
            w[2] = P.tz.strip(e2 * P.js);
            if constexpr (KIND == ABG_BP_STRIP_TAU) {
                w[0] = w[0] >= P.thr ? w[0] : T(0);
                w[1] = w[1] >= P.thr ? w[1] : T(0);
                w[2] = w[2] >= P.thr ? w[2] : T(0);
            }
        }
        return fma(w[0], win[k0], fma(w[1], win[k0 + 1], w[2] * win[k0 + 2]));
    };

    T acc[kPixPerLane] = {};
    __syncthreads();
    fetch(0);
    setup(0);
    if (n_rounds > 1) fetch(1);
    __syncthreads();
    load(0);
    for (int r = 0; r < n_rounds; ++r) {
        const int na = min(AB, n_ang - r * AB);
        __syncthreads();
        store();
        if (r + 1 < n_rounds) {
            setup(r + 1);
            if (r + 2 < n_rounds) fetch(r + 2);
        }
        __syncthreads();
        if (r + 1 < n_rounds) load(r + 1);
        for (int t = wave; t < na; t += kBackWaves) {
            const BackStageV<T> P = L.prm[r & 1][t];
            const T u0 = fma(ftx, P.cu, fma(fty, P.su, P.f));
            acc[0] += tap(L.win[t], u0, P);
#pragma unroll
            for (int j = 1; j < kPixPerLane; ++j) acc[j] += tap(L.win[t], fma(T(j), P.su4, u0), P);
        }
    }
    tile_store<T, PAD>(acc, L.part, T(1), x, N, c0, r0, xr, xc, S);
}

}  // namespace
}  // namespace abg
