// Matrix-free 2-D parallel-beam projectors for gfx950.
//
//  forward  y = A x : line model (Sec. 6.1), one thread per ray; the strip and
//           interpolation (Joseph) models of Sec. 6.1 walk the same bands. A ray crosses each
//           band of pixels along its major axis (rows when |cos| >= |sin|, else columns)
//           in a segment of length 1/p that spans at most two pixels; the kernel walks
//           the bands and splits the segment at the pixel edge it crosses, i.e. it
//           computes Siddon's exact intersection lengths band by band. Adjacent lanes
//           are adjacent rays of one angle, so every band read touches a contiguous run
//           of one image row; steep rays read the row-major copy, flat rays a transposed
//           copy, both zero-padded so that no per-tap bounds test is needed.
//  back     x = B y (unmatched, linear interpolation on the detector) or x = A^T y,
//           pixel-driven: a block owns a 16 x 16 tile, each lane 4 of its pixels, and the
//           eight waves split the angles. For a round of 64 angles the tile's detector
//           footprint (at most 32 bins per angle) is staged in LDS; every pixel then
//           reads its two taps per angle from LDS, and the eight wave partials are summed
//           in a fixed order at the end. Its output can go straight into the forward
//           projector's padded copies (AB-GMRES applies A right after B).
#include <hip/hip_ext.h>

#include <atomic>
#include <mutex>

#include "back_body.h"
#include "fwd_body.h"

namespace abg {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void pad_transpose_kernel(const T *__restrict__ x,
                                                            T *__restrict__ xr,
                                                            T *__restrict__ xc, int N, int S,
                                                            const DevState *st, int k)
{
    __shared__ PadLds<T> lds;
    if (halted(st, k)) return;
    pad_transpose_tile(x, xr, xc, N, S, blockIdx.x * 32, blockIdx.y * 32, lds);
}

template <typename T>
__global__ void pad_zero_kernel(T *__restrict__ xr, T *__restrict__ xc, int N, int S,
                                const DevState *st, int k)
{
    if (halted(st, k)) return;
    pad_zero_item(xr, xc, N, S, blockIdx.x * blockDim.x + threadIdx.x);
}

// Block shape of the forward projectors: a block's four waves take 2^lg_apb consecutive
// angles and 64 * 4 / 2^lg_apb consecutive rays of each (block (x, y): angles from
// y * 2^lg_apb, rays from x times that width). Every wave walks its own rays; with several
// angles per block the waves of a block walk nearly the same image rows at nearly the
// same time (adjacent angles cross the same pixels), which keeps those rows in L2 while
// they are reused. Waves past the last angle leave at once.
struct FwdShape {
    int lg_apb;
    __device__ int wave_angle(int wave) const { return blockIdx.y * (1 << lg_apb) + (wave >> (2 - lg_apb)); }
    __device__ int lane_ray(int wave) const
    {
        const int rays = kFwdBlock >> lg_apb;
        return blockIdx.x * rays + (wave & ((4 >> lg_apb) - 1)) * 64 + ((int)threadIdx.x & 63);
    }
};

template <typename T>
__global__ __launch_bounds__(kFwdBlock) void forward_kernel(
    const T *__restrict__ xr, const T *__restrict__ xc, T *__restrict__ y,
    const AngleParams *__restrict__ ang, int N, int S, int n_ang, int n_det, double ds,
    double s0, const DevState *st, int k, FwdShape sh)
{
    if (halted(st, k)) return;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int a = sh.wave_angle(wave);
    if (a >= n_ang) return;
    forward_ray(xr, xc, y, ang, a, sh.lane_ray(wave), N, S, n_det, ds, s0);
}

// Line model, four angles per block: a share of the blocks (stage_eighths of every 8,
// spread over the grid by a hash of the block index) walk with their band rows staged in
// LDS, the others take their taps straight from the image copies.
template <typename T>
__global__ __launch_bounds__(kFwdBlock) void forward_mixed_kernel(
    const T *__restrict__ xr, const T *__restrict__ xc, T *__restrict__ y,
    const AngleParams *__restrict__ ang, int N, int S, int n_ang, int n_det, double ds,
    double s0, const DevState *st, int k, int stage_eighths)
{
    if (halted(st, k)) return;
    __shared__ FwdStageLds<T> lds;
    const unsigned b = blockIdx.y * gridDim.x + blockIdx.x;
    if ((int)((b * 0x9E3779B1u) >> 29) < stage_eighths) {
        forward_block_staged(xr, xc, y, ang, blockIdx.y * 4, blockIdx.x * 64, N, S, n_ang, n_det,
                             ds, s0, lds);
        return;
    }
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int a = blockIdx.y * 4 + wave;
    if (a >= n_ang) return;
    forward_ray(xr, xc, y, ang, a, blockIdx.x * 64 + ((int)threadIdx.x & 63), N, S, n_det, ds, s0);
}

// Strip (MODEL = ABG_FP_STRIP) and interpolation (ABG_FP_JOSEPH) models.
template <typename T, int MODEL>
__global__ __launch_bounds__(kFwdBlock) void forward_model_kernel(
    const T *__restrict__ xr, const T *__restrict__ xc, T *__restrict__ y,
    const AngleParams *__restrict__ ang, int N, int S, int n_ang, int n_det, double ds,
    double s0, const DevState *st, int k, FwdShape sh)
{
    if (halted(st, k)) return;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int a = sh.wave_angle(wave);
    if (a >= n_ang) return;
    const int i = sh.lane_ray(wave);
    if constexpr (MODEL == ABG_FP_STRIP)
        forward_ray_strip(xr, xc, y, ang, a, i, N, S, n_det, ds, s0);
    else
        forward_ray_joseph(xr, xc, y, ang, a, i, N, S, n_det, ds, s0);
}

// 64 angles staged per round: the smaller LDS footprint lets more blocks share a CU
// (measured faster than 128 on large images, equal on small ones).
constexpr int kSingleAngBlock = 64;

// PAD: x is the forward projector's scratch (padded copies written directly).

// Transposes of the strip and interpolation models (KIND ABG_BP_STRIP_T / _JOSEPH_T) and
// the thresholded strip transpose (ABG_BP_STRIP_TAU, entries below tau_thr dropped).
template <typename T, int KIND, bool PAD>
__global__ __launch_bounds__(kBackThreads) void back_model_kernel(
    const T *__restrict__ y, T *__restrict__ x, const AngleParams *__restrict__ ang, int N,
    int n_ang, int n_det, double ds, double s0, double tau_thr, const DevState *st, int k)
{
    __shared__ BackLdsV<T, kSingleAngBlock> lds;
    if (halted(st, k)) return;
    const int S = N + 2 * kPad;
    back_tile_v<T, KIND, kSingleAngBlock, PAD>(y, x, ang, N, n_ang, n_det, ds, s0,
                                               blockIdx.x * kTile, blockIdx.y * kTile, lds, x,
                                               x + (size_t)N * S, S, tau_thr);
}

// WY: the sinogram's bytes fit a 31-bit offset (window loads through one buffer resource).
template <typename T, bool ADJ, bool PAD, bool WY>
__global__ __launch_bounds__(kBackThreads, (kBackMinWaves<T, ADJ>)) void back_kernel(
    const T *__restrict__ y, T *__restrict__ x, const AngleParams *__restrict__ ang, int N,
    int n_ang, int n_det, double ds, double s0, const DevState *st, int k)
{
    __shared__ BackLds<T, kSingleAngBlock> lds;
    if (halted(st, k)) return;
    const int S = N + 2 * kPad;
    back_tile<T, ADJ, kSingleAngBlock, PAD, WY>(y, x, ang, N, n_ang, n_det, ds, s0,
                                                blockIdx.x * kTile, blockIdx.y * kTile, lds, x,
                                                x + (size_t)N * S, S);
}

// x == nullptr: the padded copies in ws already hold the input.
template <typename T>
hipError_t forward_t(const Geometry &g, const void *x, void *y, void *ws, hipStream_t s,
                     const DevState *st, int k, bool pads_zero)
{
    const int N = g.N, S = g.padded_stride();
    T *xr = static_cast<T *>(ws);
    T *xc = xr + (size_t)N * S;
    if (x) {
        dim3 tgrid((N + 31) / 32, (N + 31) / 32);
        pad_transpose_kernel<T><<<tgrid, 256, 0, s>>>(static_cast<const T *>(x), xr, xc, N, S, st, k);
        if (!pads_zero) {
            const int npad = 2 * N * 2 * kPad;
            pad_zero_kernel<T><<<(npad + 255) / 256, 256, 0, s>>>(xr, xc, N, S, st, k);
        }
    }
    const FwdShape sh{fwd_lg_angles_per_block(g)};
    const int apb = 1 << sh.lg_apb, rays = kFwdBlock >> sh.lg_apb;
    dim3 grid((g.n_det + rays - 1) / rays, (g.n_ang + apb - 1) / apb);
    const double s0 = -0.5 * (g.n_det - 1) * g.ds;
    const int stage = fwd_stage_eighths(g, sizeof(T) == 8 ? ABG_F64 : ABG_F32);
    if (sh.lg_apb == 2 && g.model == ABG_FP_LINE && stage > 0) {
        ProfScope ps(kProfFwd, s, st ? k : 0, true);
        hipExtLaunchKernelGGL(forward_mixed_kernel<T>, grid, dim3(kFwdBlock), 0, s, ps.e0, ps.e1, 0,
                              (const T *)xr, (const T *)xc, static_cast<T *>(y),
                              (const AngleParams *)g.dev, N, S, g.n_ang, g.n_det, g.ds, s0, st, k,
                              stage);
        return hipGetLastError();
    }
    {
        // timed at the kernel's own start and end when profiling is on
        ProfScope ps(kProfFwd, s, st ? k : 0, true);
        auto fn = g.model == ABG_FP_STRIP    ? forward_model_kernel<T, ABG_FP_STRIP>
                  : g.model == ABG_FP_JOSEPH ? forward_model_kernel<T, ABG_FP_JOSEPH>
                                             : forward_kernel<T>;
        hipExtLaunchKernelGGL(fn, grid, dim3(kFwdBlock), 0, s, ps.e0, ps.e1, 0,
                              (const T *)xr, (const T *)xc, static_cast<T *>(y),
                              (const AngleParams *)g.dev, N, S, g.n_ang, g.n_det, g.ds, s0, st,
                              k, sh);
    }
    return hipGetLastError();
}

template <typename T, bool PAD>
hipError_t back_t(const Geometry &g, int kind, const void *y, void *x, hipStream_t s,
                  const DevState *st, int k)
{
    dim3 grid((g.N + kTile - 1) / kTile, (g.N + kTile - 1) / kTile);
    const double s0 = -0.5 * (g.n_det - 1) * g.ds;
    ProfScope ps(kProfBack, s, st ? k : 0, true);
    if (kind == ABG_BP_STRIP_T || kind == ABG_BP_JOSEPH_T || kind == ABG_BP_STRIP_TAU) {
        auto fn = kind == ABG_BP_STRIP_T    ? back_model_kernel<T, ABG_BP_STRIP_T, PAD>
                  : kind == ABG_BP_JOSEPH_T ? back_model_kernel<T, ABG_BP_JOSEPH_T, PAD>
                                            : back_model_kernel<T, ABG_BP_STRIP_TAU, PAD>;
        hipExtLaunchKernelGGL(fn, grid, dim3(kBackThreads), 0, s, ps.e0, ps.e1, 0,
                              static_cast<const T *>(y), static_cast<T *>(x),
                              (const AngleParams *)g.dev, g.N, g.n_ang, g.n_det, g.ds, s0,
                              g.tau_thr, st, k);
        return hipGetLastError();
    }
    const bool wy = sinogram_fits_offset(g.m(), sizeof(T));
    auto fn = kind == ABG_BP_ADJ ? (wy ? back_kernel<T, true, PAD, true> : back_kernel<T, true, PAD, false>)
                                 : (wy ? back_kernel<T, false, PAD, true> : back_kernel<T, false, PAD, false>);
    hipExtLaunchKernelGGL(fn, grid, dim3(kBackThreads), 0, s, ps.e0, ps.e1, 0,
                          static_cast<const T *>(y), static_cast<T *>(x),
                          (const AngleParams *)g.dev, g.N, g.n_ang, g.n_det, g.ds, s0, st, k);
    return hipGetLastError();
}

}  // namespace

namespace {
std::atomic<int> g_fwd_force_lg{-1};
}  // namespace


// Angles per block of the forward projectors (log2), from measurements on gfx950 (all
// shapes give the same bits). Four angles per block pay above N = 512 (640^2 x 720
// angles x 907 bins: 244 us with one angle per block, 177 with four): the 4 MB L2 of
// an XCD holds only about three band steps of the rows its resident waves read, so rows
// are reused only by waves walking nearly the same rows at nearly the same time -- the
// waves of one block at adjacent angles (FP64: 9% faster at 768^2, 27% at 2048^2, 42% at
// 1536^2; FP32 1-3%). Smaller images stay in L2 anyway; there one angle per block is
// faster (its rays share each band's cache lines within a wave) unless the last block of
// each angle leaves more lanes idle than blocks of two angles would (n_det = 363: 512
// lanes against 384, two angles 6-8% faster).
int fwd_lg_angles_per_block(const Geometry &g)
{
    const int forced = g_fwd_force_lg.load(std::memory_order_relaxed);
    if (forced >= 0) return forced;
    if (g.N > 512) return 2;
    const long long lanes1 = (g.n_det + 255LL) / 256 * 256, lanes2 = (g.n_det + 127LL) / 128 * 128;
    return lanes2 < lanes1 ? 1 : 0;
}

void fwd_force_block_shape(int lg_apb) { g_fwd_force_lg.store(lg_apb >= 0 && lg_apb <= 2 ? lg_apb : -1); }

namespace {
std::atomic<int> g_fwd_stage{-1};
}  // namespace
// Eighths of the four-angle forward blocks (line model) that stage their band rows in
// LDS, from measurements on gfx950 (all shares give the same bits; times per apply at
// 0 / 2 / 3 eighths): FP32 three eighths (2048^2 x 1800 angles 3.10 / 2.77 / 2.72 ms,
// 1024^2 x 900 0.45 / 0.41 / 0.41 ms, 640^2 x 720 177 / 166 / 161 us, 256^2 x 360 50 / 43
// / 42 us, 2048^2 x 600 1.16 / 1.08 / 1.08 ms). FP64, whose gathers return twice the
// bytes: two eighths at 1024^2 (0.47-0.53 / 0.44-0.47 ms), three below (640^2 x 720 190 /
// 174 / 175 us, 384^2 x 600 80 / 79 / 74, 256^2 x 360 53 / 52 / 43), where the four
// angles of a block stay close (N times the angle step at most 4 px; 2048^2 x 600, at
// 10.7, 1.33-1.37 / 1.41-1.42 ms), and none above 1024 (2048^2 x 1800 3.15-3.23 /
// 3.10-3.18 / 3.20 ms, within what boxes differ by). The engine's forward items take the
// FP32 / FP64 rule without the geometry.
int fwd_stage_eighths(int dtype)
{
    const int forced = g_fwd_stage.load(std::memory_order_relaxed);
    if (forced >= 0) return forced;
    return dtype == ABG_F64 ? 0 : 3;
}
int fwd_stage_eighths(const Geometry &g, int dtype)
{
    const int forced = g_fwd_stage.load(std::memory_order_relaxed);
    if (forced >= 0) return forced;
    if (dtype != ABG_F64) return 3;
    if (g.N > 1024) return 0;
    // mean step between listed angles (degrees), in radians
    const double step = g.n_ang > 1 ? std::fabs(g.theta.back() - g.theta.front()) / (g.n_ang - 1) *
                                          (3.14159265358979323846 / 180.0)
                                    : 1.0;
    if (g.N * step > 4.0) return 0;
    return g.N >= 1024 ? 2 : 3;
}
void fwd_force_stage_eighths(int e) { g_fwd_stage.store(e >= 0 && e <= 8 ? e : -1); }

size_t fp_workspace_bytes(const Geometry &g, int dtype)
{
    return align256(2 * (size_t)g.N * g.padded_stride() * dtype_size(dtype));
}

hipError_t launch_forward(const Geometry &g, int dtype, const void *x, void *y, void *ws,
                          hipStream_t s, const DevState *st, int k, bool pads_zero)
{
    return dtype == ABG_F64 ? forward_t<double>(g, x, y, ws, s, st, k, pads_zero)
                            : forward_t<float>(g, x, y, ws, s, st, k, pads_zero);
}

hipError_t launch_back(const Geometry &g, int kind, int dtype, const void *y, void *x,
                       hipStream_t s, const DevState *st, int k)
{
    return dtype == ABG_F64 ? back_t<double, false>(g, kind, y, x, s, st, k)
                            : back_t<float, false>(g, kind, y, x, s, st, k);
}

hipError_t launch_back_staged(const Geometry &g, int kind, int dtype, const void *y, void *ws,
                              hipStream_t s, const DevState *st, int k)
{
    return dtype == ABG_F64 ? back_t<double, true>(g, kind, y, ws, s, st, k)
                            : back_t<float, true>(g, kind, y, ws, s, st, k);
}

hipError_t launch_forward_staged(const Geometry &g, int dtype, void *y, void *ws, hipStream_t s,
                                 const DevState *st, int k)
{
    return dtype == ABG_F64 ? forward_t<double>(g, nullptr, y, ws, s, st, k, true)
                            : forward_t<float>(g, nullptr, y, ws, s, st, k, true);
}

// ---- forward projection without a caller workspace ------------------------------------
// The two padded copies live in a file-scope device array instead. In host code the
// array's name is only a host-side stand-in: every use goes through the device address
// that hipGetSymbolAddress returns, looked up once per device (each device holds its own
// copy of the array) on the first call there.
namespace {
constexpr size_t kStaticScratchBytes = size_t(72) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

size_t fp_static_scratch_bytes() { return kStaticScratchBytes; }

int fp_apply_static(const Geometry &g, int dtype, const void *x, void *y, hipStream_t s)
{
    if (fp_workspace_bytes(g, dtype) > kStaticScratchBytes) return ABG_ENOMEM;
    void *ptr = nullptr;
    if (scratch_address(&ptr) != hipSuccess) return ABG_EHIP;
    ProfSuppress no_events;
    // pads_zero = false: the padding is cleared by a kernel on every call, whatever an
    // earlier call left in the array
    return launch_forward(g, dtype, x, y, ptr, s, nullptr, 0, false) == hipSuccess ? ABG_OK
                                                                                 : ABG_EHIP;
}

}  // namespace abg
