// Internal declarations shared by the HIP translation units of libabgmres.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/abgmres.h"
#include "geometry.h"
#include "group_budget.h"

namespace abg {

// bf16 storage: raw 16-bit pattern, round-to-nearest-even on the way in.
struct bf16 {
    uint16_t bits;
};

struct DevState;

inline size_t dtype_size(int t) { return t == ABG_F64 ? 8 : (t == ABG_F32 ? 4 : 2); }
inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// ---- launchers (projectors.hip) ------------------------------------------------------
size_t fp_workspace_bytes(const Geometry &g, int dtype);
// `st`/`k`: when st is given, the launch is part of Arnoldi step k and returns at once
// if the solve is halted.
// `pads_zero`: the caller guarantees that the padding columns of ws are already zero.
hipError_t launch_forward(const Geometry &g, int dtype, const void *x, void *y, void *ws,
                          hipStream_t s, const DevState *st = nullptr, int k = 0,
                          bool pads_zero = false);
hipError_t launch_back(const Geometry &g, int kind, int dtype, const void *y, void *x,
                       hipStream_t s, const DevState *st = nullptr, int k = 0);
// The back projection written into the forward projector's scratch ws (its padded copies,
// whose padding must already be zero), and the forward projection of what ws holds: an
// A-after-B pair without the copy step.
hipError_t launch_back_staged(const Geometry &g, int kind, int dtype, const void *y, void *ws,
                              hipStream_t s, const DevState *st = nullptr, int k = 0);
hipError_t launch_forward_staged(const Geometry &g, int dtype, void *y, void *ws, hipStream_t s,
                                 const DevState *st = nullptr, int k = 0);

// ---- Krylov kernels (krylov.hip) -----------------------------------------------------
// Scalars of one solve, in device memory. Per-step kernels of step k return at entry
// when the solve is halted: a stop raised by an earlier step, or an Arnoldi breakdown
// at an earlier step. The host reads a copy after every step.
struct DevState {
    double beta;         // ||r_0||
    double qnorm0;       // ||q_k|| before orthogonalisation
    double hnext;        // h_{k+1,k}
    double ls;           // |g_{k+1}|: GMRES residual of the small least-squares problem
    double res;          // norm written by the last residual reduction
    double ncp;          // d_k
    double ncp_prev;     // d_{k-1}
    double dp_thr;       // DP candidate threshold tau*||e||*(1+slack); 0 without DP
    double err;          // ||x_k - x_ref|| (error-history runs only)
    int k;               // step that last completed its Givens update
    int bd_k;            // step at which h_{k+1,k} fell below the breakdown bound (0: none)
    int error;           // sticky: 1 grid-barrier timeout, 2 non-finite norm, 4 singular R
    int stop;            // raised by the last kernel of a step: later steps return at entry
    int stop_k;          // step that raised it
    int stop_reason;     // kStop*
    // batched solves only
    int kcur;            // step being run this round (0: the instance sits it out)
    int active;          // initialised, with beta > 0
    int done;            // final: x holds x_{k_sel}, lit = ||b - A x||, status set
    int k_sel;           // step whose iterate x holds
    int status;          // ABG_* status of the finished instance
    int n_lit;           // DP candidates checked with the explicit residual
    int gen;             // admission counter of the slot (tells a reused slot's copies apart)
    double lit;          // ||b - A x|| of the last iterate formed
};
enum { kStopNone = 0, kStopDP = 1, kStopNCP = 2, kStopError = 3, kStopZero = 4 };

#ifdef __HIPCC__
// A pointer read from memory (a descriptor field) is a generic pointer to the compiler,
// which then emits flat loads through it. Reading the field as a global-address-space
// pointer and converting that value to a generic one lets the compiler prove the target
// is global memory and use global loads (cheaper addressing, and not counted against
// LDS traffic).
template <typename T, typename F> __device__ inline T *gfield(const F &field)
{
    static_assert(sizeof(F) == sizeof(void *), "pointer field");
#if defined(__HIP_DEVICE_COMPILE__)
    using GP = __attribute__((address_space(1))) T *;
    return (T *)(*reinterpret_cast<const GP *>(&field));
#else
    return (T *)field;
#endif
}

// True when per-step kernels of step k must not run.
__device__ inline bool halted(const DevState *st, int k)
{
    if (!st) return false;
    const volatile DevState *v = st;
    return v->stop != 0 || (v->bd_k != 0 && v->bd_k < k) || v->error != 0;
}
#endif

// Vectors that Gram-Schmidt reads or writes (q, the basis columns, the current vector) are
// allocated with a length rounded up to a multiple of kVecPad elements, zero past their
// logical length, so that every register tile of the MGS kernels lies inside them.
constexpr long long kVecPad = 16384;
// Data format word of a raw gfx9 buffer resource (projector loads through
// __builtin_amdgcn_make_buffer_rsrc: offsets past the resource's size read zero).
constexpr int kRawBufferFlags = 0x00020000;
// The back projectors read the sinogram through one buffer resource when its bytes fit a
// 31-bit offset (batched problems must; single applies fall back to clamped addresses).
inline bool sinogram_fits_offset(long long m, size_t elem) { return (size_t)m * elem < 0x80000000ull; }
// Longer vectors may not fit the registers of one resident block group: their solves
// carry an FP64 scratch copy of q_k for the streaming Gram-Schmidt variant.
constexpr long long kRegMaxL = 2 * 1024 * 1024;

struct MgsLaunch {
    int tx, tv;                  // dtypes of q / cur and of the basis
    const void *q;               // q_k, L elements of tx
    const void *V;               // basis, vector i at V + i*ldv elements
    size_t ldv;
    int k;                       // orthogonalise against w_1..w_k (k may be 0)
    long long L;
    double *hcol;                // out: k+1 values h_{1,k}..h_{k+1,k}
    void *vout;                  // out: w_{k+1} (tv), at V + k*ldv
    void *cur;                   // out: w_{k+1} converted back to tx
    double *partials;            // reduction slot tables: 2 x rows x G doubles
    int rows;                    // rows per table (>= k + 3 for every step of the solve)
    unsigned *ticket;            // zeroed counter of this step: hands out block ranks
    double *q64;                 // FP64 scratch of L elements (needed when L > kRegMaxL)
    DevState *st;
    double bd_rel;               // breakdown: h_{k+1,k} <= bd_rel * ||q_k||
    int step;                    // Arnoldi step (0: the initial normalisation)
    // single solves only (zero otherwise)
    int set_beta;                // step 0: beta = h_{1,0}, or the zero-right-hand-side stop
    // step k >= 1: the Givens update of column k follows in the same launch (giv_H null:
    // none); arguments as for launch_givens, beta read from st; snap as for launch_combine
    double *giv_H, *giv_R, *giv_cs, *giv_sn, *giv_g, *giv_y, *giv_rho;
    int giv_ld;
    DevState *snap;
    // strictly lower triangle of the basis Gram matrix (gram_entries(k_max) doubles),
    // kept across the steps of one solve; set: steps 2..64 run the low-synchronisation
    // form (rows >= 2 k_max + 3); null: plain MGS
    double *gram;
};
constexpr int kMaxGrid = 2048;
// Largest Arnoldi step that runs the low-synchronisation form of Gram-Schmidt, and the
// size of the packed Gram triangle it keeps (rows 0..min(k_max, kIcwyMaxK) - 1).
constexpr int kIcwyMaxK = 64;
constexpr size_t gram_entries(int k_max)
{
    const size_t r = (size_t)(k_max < kIcwyMaxK ? k_max : kIcwyMaxK);
    return r * (r - 1) / 2 + 1;
}
hipError_t launch_mgs(const MgsLaunch &a, hipStream_t s);

// out = base_coef*base + sum_{j<kk} sgn*coef[j]*V_j  (FP64 accumulation). With `norm`
// set, ||out||_2 is reduced in a fixed order by the last block to finish and written to
// *norm; when st is given the launch belongs to step k (halt check) and, if
// st->dp_thr > 0 and ||out|| <= dp_thr, raises the DP stop for step k. `count` is a
// zeroed counter that the last block resets. `snap` (norm and st given): a device-visible
// copy of *st is written there once the launch is over (also when the step is halted).
hipError_t launch_combine(int tout, const void *base, double base_coef, int tv, const void *V,
                          size_t ldv, int kk, const double *coef, double sgn, void *out,
                          long long L, double *partials, unsigned *count, double *norm,
                          DevState *st, int k, hipStream_t s, DevState *snap = nullptr);
// out = a - b with partial sums of out^2.
hipError_t launch_sub_norm(int t, const void *a, const void *b, void *out, long long L,
                           double *partials, int *nblocks, hipStream_t s);
// dst = sqrt(sum partials[0..nb)) (fixed order, one block).
hipError_t launch_reduce_sqrt(const double *partials, int nb, double *dst, hipStream_t s);
// Givens update of column k of H, y_k into y (k entries), and rho = beta e_1 - H_k y_k
// when rho is given (beta read on the device). `snap`: as for launch_combine.
hipError_t launch_givens(double *H, int ld, double *R, double *cs, double *sn, double *g,
                         double *y, double *rho, const double *beta, int k, DevState *st,
                         hipStream_t s, DevState *snap = nullptr);
// st->beta = st->hnext after the initial normalisation, or the zero-right-hand-side stop.
hipError_t launch_set_beta(DevState *st, hipStream_t s);
// Clears the stop flag (after a DP candidate that the explicit residual rejected).
hipError_t launch_clear_stop(DevState *st, hipStream_t s);
void set_mgs_target_blocks(int blocks);
// Single solves use the streaming Gram-Schmidt variant whenever their workspace has its
// scratch (vectors longer than kRegMaxL), not only when the register tile does not fit.
void set_mgs_force_stream(int on);
hipError_t launch_fill_u32(unsigned *p, size_t n, unsigned v, hipStream_t s);
hipError_t launch_fill_f64(double *p, size_t n, double v, hipStream_t s);
// One range of a fused initialisation: n 32-bit words at p; the first n_src are copied
// from src, the others set to the 64-bit pattern (lo, hi) (even words lo, odd words hi,
// so p is 8-byte aligned when lo != hi). Ranges must not overlap.
struct FillRange {
    void *p;
    const void *src;
    unsigned long long n, n_src;
    unsigned lo, hi;
};
constexpr int kMaxFill = 12;
// All ranges in one launch; with init, *st = *init as well.
hipError_t launch_init_fill(const FillRange *r, int n, const DevState *init, DevState *st,
                            hipStream_t s);
// Bit pattern of an empty MGS reduction slot.
unsigned long long slot_empty_bits();
// Marks MGS reduction slots empty (n doubles).
hipError_t launch_clear_slots(double *p, size_t n, hipStream_t s);
hipError_t launch_axpy_inplace(int t, void *x, const void *x0, long long L, hipStream_t s);

// ---- NCP (ncp.hip) ------------------------------------------------------------------
size_t ncp_scratch_bytes(const Geometry &g);
// Frees the geometry's periodogram tables (abg_destroy_geometry).
void ncp_release(Geometry &g);
// Process-wide: periodograms by Goertzel's recurrence for every row length (tests).
void ncp_force_goertzel(int on);
// Process-wide: forward projector block shape, 2^lg_apb angles per block (0..2), or -1 for
// the automatic choice (tests and measurements).
void fwd_force_block_shape(int lg_apb);
// Forward projector block shape (log2 of the angles per block of 256 threads) for a
// geometry: the choice single solves make, or the forced one.
int fwd_lg_angles_per_block(const Geometry &g);
int fwd_stage_eighths(int dtype);
int fwd_stage_eighths(const Geometry &g, int dtype);
void fwd_force_stage_eighths(int eighths);
// d_k of the residual r into st->ncp; raises the NCP stop for step k when k >= 2 and
// d_k > d_{k-1}. `snap`: as for launch_combine.
hipError_t launch_ncp(const Geometry &g, int t, const void *r, double *scratch, DevState *st,
                      int k, hipStream_t s, DevState *snap = nullptr);

// ---- LSQR / LSMR (lsq.hip) -------------------------------------------------------------
// FP64 scalars of the recurrences (device memory). alpha, beta: alpha_k, beta_k of the
// current step; alpha_n, beta_n: alpha_{k+1}, beta_{k+1} once computed.
struct LsqScalars {
    double alpha, beta, alpha_n, beta_n;
    double rhobar, phibar;                                          // LSQR
    double alphabar, zetabar, rho_prev, rhobar_prev, cbar, sbar;    // LSMR
    double theta, hcoef, xcoef;                                     // LSMR
};
// u <- t - (alpha/beta) u, beta_n = ||u||; with ah: ah <- t - (theta/rho_prev) ah.
hipError_t launch_lsq_u(int t, void *u, const void *tv, void *ah, long long m, LsqScalars *S,
                        double *partials, unsigned *count, DevState *st, int k, hipStream_t s);
// v <- s/beta_n - beta_n v, alpha_n = ||v||.
hipError_t launch_lsq_v(int t, void *v, const void *sv, long long n, LsqScalars *S,
                        double *partials, unsigned *count, DevState *st, int k, hipStream_t s);
// xprev (optional): receives the previous iterate
hipError_t launch_lsqr_x(int t, void *x, void *xprev, void *w, void *v, long long n,
                         LsqScalars *S, unsigned *count, DevState *st, int k, DevState *snap,
                         hipStream_t s);
hipError_t launch_lsmr_x(int t, void *x, void *xprev, void *h, void *hbar, void *v, long long n,
                         LsqScalars *S, unsigned *count, DevState *st, int k, hipStream_t s);
hipError_t launch_lsmr_r(int t, const void *ah, void *ahbar, void *r, long long m, LsqScalars *S,
                         double *partials, unsigned *count, DevState *st, int k, DevState *snap,
                         hipStream_t s);
hipError_t launch_lsq_start(int t, void *v, void *w, void *hbar, long long n, LsqScalars *S,
                            unsigned *count, DevState *st, int lsmr, hipStream_t s);

// ---- solvers (solver.hip) -----------------------------------------------------------
size_t solver_workspace_bytes(const Geometry &g, int method, int k_max, abg_precision p,
                              abg_stop st);
// LSQR (method ABG_METHOD_LSQR) or LSMR (ABG_METHOD_LSMR) with A the geometry's model and
// its exact transpose.
size_t lsq_workspace_bytes(const Geometry &g, int method, int dtype);
// x_ref (device, n elements) and err_hist (host, k_max entries), both optional together:
// err_hist[k-1] = ||x_k - x_ref|| for every step k performed.
int run_lsq(const Geometry &g, int method, const void *b, const void *x0, void *x, int k_max,
            abg_stop st, int dtype, void *ws, size_t ws_bytes, abg_info *info,
            const void *x_ref, double *err_hist, hipStream_t s);
int run_solver(const Geometry &g, int method, int kind, const void *b, const void *x0,
               void *x, int k_max, abg_stop st, abg_precision p, void *ws, size_t ws_bytes,
               abg_info *info, hipStream_t s);
// After run_solver on ws with the same arguments: err[k-1] = ||x_k - x_ref|| for
// k = 1..k_done, each iterate rebuilt from the stored basis and small-problem solutions.
int gmres_error_history(const Geometry &g, int method, int kind, int k_max, abg_stop st,
                        abg_precision p, void *ws, size_t ws_bytes, const void *x0,
                        const void *x_ref, int k_done, double *err, hipStream_t s);

// ---- one problem of the batched engine (solver.hip) ------------------------------------
// Buffers inside a solve's workspace (the same layout as a single solve).
struct InstanceView {
    void *V, *Z, *cur, *q, *rb0, *tm, *tn, *fpws;
    double *H, *R, *cs, *sn, *g, *Y, *rho, *part, *mgs_part, *q64;
    unsigned *count;
    long long L, ldv, mp, np;
    int part_cap;                 // doubles in part
    int mgs_rows;                 // rows per MGS slot table
    long long mgs_part_cap;       // doubles in mgs_part (two tables)
};
InstanceView instance_view(const Geometry &g, int method, int k_max, abg_precision p,
                           abg_stop st, void *ws);
// Enqueues the initialisation (clears, r0, MGS step 0 into *dst); no host wait.
int instance_init(const Geometry &g, int method, int kind, int k_max, abg_stop st,
                  abg_precision p, void *ws, const void *b, const void *x0, DevState *dst,
                  hipStream_t s);
// Enqueues x = x_k (k = 0: x0 or zero) and ||b - A x|| into *lit; no host wait.
int instance_form_x(const Geometry &g, int method, int kind, int k_max, abg_stop st,
                    abg_precision p, void *ws, int k, const void *b, const void *x0, void *x,
                    DevState *dst, double *lit, hipStream_t s);

// ---- batched engine (batch.hip) ---------------------------------------------------------
struct Engine;
int engine_create(abg_precision p, int max_slots, hipStream_t s, Engine **out);
void engine_destroy(Engine *e);
int engine_submit(Engine *e, const Geometry &g, const abg_request &r);
int engine_step(Engine *e, int *n_running);
int engine_poll(Engine *e, long long *tags, int *status, int max, int *n);
int engine_pending(const Engine *e);
int engine_set_tiles(Engine *e, int rays, int ang_block, int sched);
int engine_get_tiles(const Engine *e, int *rays, int *ang_block, int *sched);
int engine_autotune(Engine *e, int reps, int *rays, int *ang_block, int *sched, double *ms);
int engine_device(const Engine *e);
hipStream_t engine_stream(const Engine *e);
int engine_precision(const Engine *e, abg_precision *p);
long long engine_rounds(const Engine *e);

// Admission of spinning Gram-Schmidt block groups (krylov.hip): the current device's
// budget, and the units a single solve's Gram-Schmidt launches hold for vectors of L
// elements (tx, tv: projector and basis dtypes; q64: the FP64 scratch of the streaming
// variant exists).
GroupBudget &device_group_budget();
hipError_t mgs_group_units(int tx, int tv, long long L, bool q64, long long *units);

// Frees the idle pooled pinned scalar slots and step events of single solves (solver.hip).
int host_release_all();

// Forward projection through the library's static device scratch instead of a caller
// workspace (projectors.hip); ABG_ENOMEM when the padded copies do not fit it.
size_t fp_static_scratch_bytes();
int fp_apply_static(const Geometry &g, int dtype, const void *x, void *y, hipStream_t s);

// ---- profiling (capi.cpp) -----------------------------------------------------------
enum ProfKind { kProfFwd = 0, kProfBack = 1, kProfMgs = 2, kProfCombine = 3, kProfNcp = 4, kProfKinds = 5 };
bool profiling_on();
// Brackets one launch with timing events when profiling is on. `step` tags launches
// that belong to an Arnoldi step of the solve running on this thread; launches of
// steps that a solve enqueued but never ran (past its stop) are dropped at its end.
// With `ext`, the caller passes e0/e1 to hipExtLaunchKernelGGL, which stamps them at the
// kernel's own start and end (when profiling is off both are null).
struct ProfScope {
    ProfScope(int kind, hipStream_t s, int step = 0, bool ext = false);
    ~ProfScope();
    int kind, step;
    hipStream_t s;
    bool ext;
    hipEvent_t e0 = nullptr, e1 = nullptr;
};
// While one of these lives, launches of the current thread are not timed (their
// ProfScope takes no events): entry points that must not create any.
struct ProfSuppress {
    ProfSuppress();
    ~ProfSuppress();
    bool prev;
};
void profile_flush();
void profile_solve_begin();
// Drops this thread's pending launches of steps > last_step (enqueued past the stop).
void profile_solve_end(int last_step);
// Drops this thread's pending launches of `step` enqueued so far (a step that was
// skipped and is about to be enqueued again).
void profile_drop_step(int step);

}  // namespace abg

struct abg_geometry {
    abg::Geometry g;
};

struct abg_engine {
    abg::Engine *e;
};
