// Matrix-free 2-D parallel-beam projectors for gfx950.
//
//  forward  y = A x : line model (Sec. 6.1), one thread per ray. A ray crosses each
//           band of pixels along its major axis (rows when |cos| >= |sin|, else columns)
//           in a segment of length 1/p that spans at most two pixels; the kernel walks
//           the bands and splits the segment at the pixel edge it crosses, i.e. it
//           computes Siddon's exact intersection lengths band by band. Adjacent lanes
//           are adjacent rays of one angle, so every band read touches a contiguous run
//           of one image row; steep rays read the row-major copy, flat rays a transposed
//           copy, both zero-padded so that no per-tap bounds test is needed.
//  back     x = B y (unmatched, linear interpolation on the detector) or x = A^T y,
//           one thread per pixel of a 16 x 16 tile. For a block of 32 angles the tile's
//           detector footprint (at most 32 bins per angle) is staged in LDS, then every
//           pixel reads its two taps per angle from LDS.
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
constexpr int kTile = 16;
constexpr int kAngBlock = 32;
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
template <typename T>
__global__ __launch_bounds__(256) void pad_transpose_kernel(const T *__restrict__ x,
                                                            T *__restrict__ xr,
                                                            T *__restrict__ xc, int N, int S)
{
    __shared__ T tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
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
__global__ void pad_zero_kernel(T *__restrict__ xr, T *__restrict__ xc, int N, int S)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int per_row = 2 * kPad;
    if (idx >= 2 * N * per_row) return;
    const int row = idx / per_row, k = idx % per_row;
    const int col = k < kPad ? k : N + k;   // [0,kPad) and [N+kPad, N+2kPad)
    T *base = row < N ? xr + (size_t)row * S : xc + (size_t)(row - N) * S;
    base[col] = T(0);
}

template <typename T>
__global__ __launch_bounds__(kFwdBlock) void forward_kernel(
    const T *__restrict__ xr, const T *__restrict__ xc, T *__restrict__ y,
    const AngleParams *__restrict__ ang, int N, int S, int n_det, double ds, double s0)
{
    const int a = blockIdx.y;
    const int i = blockIdx.x * kFwdBlock + threadIdx.x;
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
        const int wr0 = wave_min_i(r0);
        const int wr1 = wave_max_i(r1);
        double lo = fma((double)wr0, P.m, lo0);
        const T *row = img + (size_t)wr0 * S;
        const double invq = P.invq, len = P.len;
        const T lenT = T(len);
        for (int r = wr0; r < wr1; ++r) {
            const double lc = fmin(fmax(lo, lo_clamp), hi_clamp);
            const double fl = floor(lc);
            const int c = (int)fl;
            // part of the band segment left of the edge at fl+1
            const T wlo = T(fmin(len, ((fl + 1.0) - lc) * invq));
            const T whi = lenT - wlo;
            acc = fma(wlo, row[c], acc);
            acc = fma(whi, row[c + 1], acc);
            lo += P.m;
            row += S;
        }
    }
    if (i < n_det) y[(size_t)a * n_det + i] = acc;
}

template <typename T>
struct alignas(16) BackStage {
    T f;       // u of the tile's reference pixel relative to the staged window start
    T cu, su;  // du per pixel step in x and in y
    T invp, half, invpq;
    int ib;    // first staged bin
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

template <typename T, bool ADJ>
__global__ __launch_bounds__(kTile *kTile) void back_kernel(
    const T *__restrict__ y, T *__restrict__ x, const AngleParams *__restrict__ ang, int N,
    int n_ang, int n_det, double ds, double s0)
{
    __shared__ T win[kAngBlock][kWin];
    __shared__ BackStage<T> prm[kAngBlock];
    const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;
    const int c0 = blockIdx.x * kTile, r0 = blockIdx.y * kTile;
    const double xref = c0 - 0.5 * N + 0.5, yref = r0 - 0.5 * N + 0.5;
    const T ftx = T(tx), fty = T(ty);
    const T dsT = T(ds);
    T acc = T(0);
    for (int a0 = 0; a0 < n_ang; a0 += kAngBlock) {
        const int na = min(kAngBlock, n_ang - a0);
        __syncthreads();
        if (threadIdx.x < na) {
            const AngleParams P = ang[a0 + threadIdx.x];
            const double cu = P.c / ds, su = P.s / ds;
            const double uref = (fma(xref, P.c, yref * P.s) - s0) / ds;
            const double umin = uref + (kTile - 1) * (fmin(cu, 0.0) + fmin(su, 0.0));
            const double ib = floor(umin) - 1.0;
            BackStage<T> st;
            st.f = T(uref - ib);
            st.cu = T(cu);
            st.su = T(su);
            st.invp = T(1.0 / P.p);
            st.half = T(0.5 * (P.p + P.q));
            st.invpq = P.axis ? T(0) : T(1.0 / (P.p * P.q));
            st.ib = (int)ib;
            st.axis = P.axis;
            prm[threadIdx.x] = st;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < na * kWin; e += kTile * kTile) {
            const int t = e / kWin, k = e % kWin;
            const int bin = prm[t].ib + k;
            win[t][k] = (bin >= 0 && bin < n_det) ? y[(size_t)(a0 + t) * n_det + bin] : T(0);
        }
        __syncthreads();
        for (int t = 0; t < na; ++t) {
            const BackStage<T> P = prm[t];
            const T u = fma(ftx, P.cu, fma(fty, P.su, P.f));
            const T fl = floor(u);
            const T w = u - fl;
            const int k = min(max((int)fl, 0), kWin - 2);
            const T v0 = win[t][k], v1 = win[t][k + 1];
            if (!ADJ) {
                acc += fma(w, v1 - v0, v0);
            } else {
                acc = fma(trapezoid(w * dsT, P), v0, acc);
                acc = fma(trapezoid((T(1) - w) * dsT, P), v1, acc);
            }
        }
    }
    const int c = c0 + tx, r = r0 + ty;
    if (r < N && c < N) x[(size_t)r * N + c] = ADJ ? acc : acc * T(1.0 / ds);
}

template <typename T>
hipError_t forward_t(const Geometry &g, const void *x, void *y, void *ws, hipStream_t s)
{
    const int N = g.N, S = g.padded_stride();
    T *xr = static_cast<T *>(ws);
    T *xc = xr + (size_t)N * S;
    dim3 tgrid((N + 31) / 32, (N + 31) / 32);
    pad_transpose_kernel<T><<<tgrid, 256, 0, s>>>(static_cast<const T *>(x), xr, xc, N, S);
    const int npad = 2 * N * 2 * kPad;
    pad_zero_kernel<T><<<(npad + 255) / 256, 256, 0, s>>>(xr, xc, N, S);
    dim3 grid((g.n_det + kFwdBlock - 1) / kFwdBlock, g.n_ang);
    const double s0 = -0.5 * (g.n_det - 1) * g.ds;
    {
        ProfScope ps(kProfFwd, s);
        forward_kernel<T><<<grid, kFwdBlock, 0, s>>>(xr, xc, static_cast<T *>(y), g.dev, N, S,
                                                     g.n_det, g.ds, s0);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t back_t(const Geometry &g, int kind, const void *y, void *x, hipStream_t s)
{
    dim3 grid((g.N + kTile - 1) / kTile, (g.N + kTile - 1) / kTile);
    const double s0 = -0.5 * (g.n_det - 1) * g.ds;
    ProfScope ps(kProfBack, s);
    if (kind == ABG_BP_ADJ)
        back_kernel<T, true><<<grid, kTile * kTile, 0, s>>>(
            static_cast<const T *>(y), static_cast<T *>(x), g.dev, g.N, g.n_ang, g.n_det, g.ds, s0);
    else
        back_kernel<T, false><<<grid, kTile * kTile, 0, s>>>(
            static_cast<const T *>(y), static_cast<T *>(x), g.dev, g.N, g.n_ang, g.n_det, g.ds, s0);
    return hipGetLastError();
}

}  // namespace

size_t fp_workspace_bytes(const Geometry &g, int dtype)
{
    return align256(2 * (size_t)g.N * g.padded_stride() * dtype_size(dtype));
}

hipError_t launch_forward(const Geometry &g, int dtype, const void *x, void *y, void *ws,
                          hipStream_t s)
{
    return dtype == ABG_F64 ? forward_t<double>(g, x, y, ws, s) : forward_t<float>(g, x, y, ws, s);
}

hipError_t launch_back(const Geometry &g, int kind, int dtype, const void *y, void *x,
                       hipStream_t s)
{
    return dtype == ABG_F64 ? back_t<double>(g, kind, y, x, s) : back_t<float>(g, kind, y, x, s);
}

}  // namespace abg
