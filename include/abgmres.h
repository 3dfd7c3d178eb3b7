/*
 * abgmres.h -- C ABI of the MI355X (gfx950) AB-GMRES / BA-GMRES reconstruction library.
 *
 * Method: Hansen, Hayami & Morikuni, "GMRES methods for tomographic reconstruction with
 * an unmatched back projector" (arXiv 2110.01481). The library solves the CT least
 * squares problem A x ~ b, b = A x_bar + e (eq. 1.1), with a forward projector A and a
 * back projector B that need not be A^T (Sec. 1), by
 *   AB-GMRES: min_u || b - A B u ||_2, x = B u          (Sec. 2, B right preconditioner)
 *   BA-GMRES: min_x || B b - B A x ||_2                  (Sec. 2, B left preconditioner)
 * following the algorithm listed in Sec. 2 (Arnoldi with modified Gram-Schmidt, the
 * (k+1) x k Hessenberg least squares problem, iterate and residual), and stops with
 * the discrepancy principle or the NCP criterion (Sec. 6.3). Steps 2..64 of a single
 * solve obtain MGS's coefficients in the inverse compact WY form (equal in exact
 * arithmetic; two grid reductions per step instead of k + 1).
 *
 * Operators (matrix-free, 2-D parallel beam; conventions, since the paper fixes none):
 *   image    N x N unit pixels centred on the origin, row-major: pixel (r, c) has
 *            index j = r*N + c and covers [c-N/2, c-N/2+1] x [r-N/2, r-N/2+1].
 *   angles   theta_a in degrees, omega_a = (cos, sin), exact 0/+-1 at multiples of 90.
 *   detector s_i = (i - (n_det-1)/2) * det_spacing; sinogram is angle-major,
 *            index a*n_det + i; ray (a,i) is the line <p, omega_a> = s_i.
 *   A        line model: A[(a,i), j] = length of ray (a,i) inside pixel j (Sec. 6.1's
 *            "line model"); a ray running exactly along a pixel edge gives half its
 *            length to each of the two pixels. Computed ray-driven on the GPU.
 *   B (HAT)  unmatched back projector: B[j,(a,i)] = max(0, 1-|u-i|)/det_spacing with
 *            u = (<c_j, omega_a> - s_0)/det_spacing, c_j the pixel centre (linear
 *            interpolation on the detector, pixel-driven; zero beyond the detector).
 *   B (ADJ)  the matched back projector A^T, for matched runs (Sec. 5).
 *   A_s      strip model (Sec. 6.1, abg_geometry_set_model): ray (a,i) is the strip of
 *            width det_spacing around s_i; weight = area of strip and pixel / det_spacing.
 *   A_i      interpolation (Joseph) model: along the ray's major axis (rows when
 *            |cos| >= |sin|) each row is interpolated linearly at the ray's crossing of
 *            its centre line, weight 1/max(|cos|,|sin|) per row.
 *   STRIP_T, JOSEPH_T  the transposes A_s^T, A_i^T (pixel-driven).
 *
 * Conventions of every entry point:
 *   - Device buffers (x, y, b, workspaces) are caller-owned device pointers on the
 *     device that was current when the geometry was created; the library never frees
 *     or keeps them past the call. The geometry handle is library-owned.
 *   - `stream` is a hipStream_t passed as void*; NULL is the legacy default stream.
 *     Apply calls are asynchronous on it; solver calls synchronise it before returning.
 *   - Return value: ABG_OK (0), a negative error or a positive informational status.
 *     No exception crosses the ABI and the library never aborts the process.
 *   - Calls are thread-safe as long as concurrent calls use distinct workspaces and
 *     output buffers. A solve's Gram-Schmidt launch needs its whole block group (256
 *     blocks for vectors of up to 2^22 elements, more for longer ones, never more than
 *     the device holds of that kernel) resident at once:
 *     solves run concurrently on several streams whose groups together exceed what the
 *     device holds can end with ABG_EDEVICE (the bounded wait) instead of completing.
 *     Many problems at once belong on one engine (below), which has no such limit.
 */
#ifndef ABGMRES_H
#define ABGMRES_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ----------------------------------------------------------------- */
#define ABG_OK 0
#define ABG_EINVAL (-1)        /* invalid argument (sizes, NULL pointer, enum value)    */
#define ABG_ENOMEM (-2)        /* workspace smaller than abg_*_workspace_bytes says      */
#define ABG_EHIP (-3)          /* a HIP runtime call failed                              */
#define ABG_ENAN (-4)          /* a norm became NaN or Inf                               */
#define ABG_EDEVICE (-5)       /* a device-side wait exceeded its bound (grid barrier)   */
#define ABG_EFULL (-6)         /* batched engine: every slot holds an unfinished problem  */
#define ABG_NOT_CONVERGED 1    /* DP never satisfied up to k_max: x_{k_max} returned     */
#define ABG_BREAKDOWN 2        /* h_{k+1,k} ~ 0: Krylov space exhausted, x_k returned    */
#define ABG_ZERO_RHS 3         /* ||r_0|| = 0: x = x_0 returned with k = 0               */

typedef enum { ABG_F64 = 0, ABG_F32 = 1, ABG_BF16 = 2 } abg_dtype;
/* Back projectors: HAT the unmatched interpolating B; ADJ = A_line^T; STRIP_T and
 * JOSEPH_T the transposes of the strip and interpolation models (unmatched pairs of
 * Sec. 6: B = A'^T with A' another model than the forward projector's); STRIP_TAU the
 * thresholded strip transpose B_tau of Sec. 6.5 (abg_geometry_set_strip_threshold). */
typedef enum {
    ABG_BP_HAT = 0,
    ABG_BP_ADJ = 1,
    ABG_BP_STRIP_T = 2,
    ABG_BP_JOSEPH_T = 3,
    ABG_BP_STRIP_TAU = 4
} abg_bp_kind;
/* Discretisation models of the forward projector A (Sec. 6.1). */
typedef enum { ABG_FP_LINE = 0, ABG_FP_STRIP = 1, ABG_FP_JOSEPH = 2 } abg_fp_model;
typedef enum { ABG_STOP_NONE = 0, ABG_STOP_DP = 1, ABG_STOP_NCP = 2 } abg_stop_kind;
typedef enum { ABG_METHOD_AB = 0, ABG_METHOD_BA = 1, ABG_METHOD_LSQR = 2, ABG_METHOD_LSMR = 3 } abg_method;

typedef struct abg_geometry abg_geometry;

/* Stopping rule (Sec. 6.3). DP: stop at the smallest k with ||b - A x_k||_2 <= tau*noise_norm
 * (tau >= 1, noise_norm = ||e||_2 > 0). NCP: normalised cumulative periodogram of each
 * sinogram row of b - A x_k, averaged over rows; stop at the first k whose distance to
 * the white-noise line is below the next one's and return x_k. NONE: run k_max steps. */
typedef struct {
    int kind;            /* abg_stop_kind */
    double tau;
    double noise_norm;
} abg_stop;

/* Arithmetic: `proj` is the dtype of projector inputs/outputs, of b, x, x0 (ABG_F64 or
 * ABG_F32); `basis` is the storage dtype of the Krylov basis (ABG_F64, ABG_F32 or
 * ABG_BF16; not wider than needed: F64 basis requires F64 proj). Dots, norms, the
 * Hessenberg matrix, Givens rotations and the small triangular solve are FP64 always. */
typedef struct {
    int proj;
    int basis;
} abg_precision;

/* Per-solve report, written on return. Arrays are caller-owned host memory of length
 * hist_len (or NULL); entry k-1 belongs to iteration k. */
typedef struct {
    int k_stop;          /* iteration whose iterate x_k was returned (0: x_0)               */
    int k_done;          /* Arnoldi steps performed                                         */
    int status;          /* same value the call returns                                    */
    int n_literal;       /* explicit ||b - A x_k|| evaluations made for the DP decision     */
    double res_norm;     /* ||b - A x||_2 of the returned x: evaluated explicitly, except   */
                         /* BA-GMRES with the NCP rule, where it is the norm of the         */
                         /* residual the rule evaluated for that iterate, b - A x_0 -       */
                         /* sum_i y_i (A w_i) from the step's stored products A w_i (equal  */
                         /* to b - A x up to the rounding of the sum; no further projection)*/
    double ncp_dist;     /* NCP distance d of the returned iterate (NCP runs)               */
    double beta;         /* ||r_0||_2                                                       */
    double *res_hist;    /* ||b - A x_k||_2 per k (DP and NCP runs), else untouched        */
    double *ls_hist;     /* || ||r_0|| e_1 - H_k y_k ||_2 (GMRES residual) per k            */
    double *ncp_hist;    /* d_k per k (NCP runs)                                            */
    int hist_len;
    double *H;           /* optional: Hessenberg matrix, (k_max+1) x k_max, column-major,   */
                         /* leading dimension k_max+1; column k-1 filled for k <= k_done    */
} abg_info;

/* ---- geometry (Table 6.1 parameters) ---------------------------------------------- */

/* Creates a parallel-beam geometry on the current HIP device.
 * N >= 1 image side; n_ang >= 1 angles: angles_deg[a] if angles_deg != NULL, else
 * ang_start_deg + a*ang_range_deg/n_ang; n_det >= 1 bins of spacing det_spacing in
 * [0.75, 64] (the matched back projector assumes at most two bins per pixel and angle).
 * Copies the angle table to device memory it owns. Returns ABG_EINVAL on bad sizes. */
int abg_create_geometry(int N, int n_ang, double ang_start_deg, double ang_range_deg,
                        const double *angles_deg, int n_det, double det_spacing,
                        abg_geometry **out);

/* Releases the geometry and its device memory. NULL is accepted. */
int abg_destroy_geometry(abg_geometry *g);

/* n = N*N (image length) and m = n_ang*n_det (sinogram length). */
int abg_geometry_sizes(const abg_geometry *g, long long *n, long long *m);

/* Forward projector model of the geometry (abg_fp_model), used by abg_fp_apply and by the
 * solvers; ABG_FP_LINE when created. The strip model needs det_spacing <= 1.4 (at most
 * four pixels per row and ray): ABG_EINVAL otherwise. Not to be changed while a solve or
 * an engine request uses the geometry. The batched engine takes line-model geometries
 * only. */
int abg_geometry_set_model(abg_geometry *g, int fp_model);
int abg_geometry_get_model(const abg_geometry *g, int *fp_model);

/* Threshold of the back projector ABG_BP_STRIP_TAU (Sec. 6.5): B_tau keeps the entries of
 * A_s^T that are >= tau * max(A_s), 0 <= tau <= 1; entries within 1e-6 * max(A_s) of the
 * threshold count as on it (kept), so that ties are decided the same way whatever the
 * rounding. The first call computes max(A_s), the largest strip-model entry of the
 * geometry, on the host (a scan of the pixel-bin pairs of the angles that can hold it)
 * and writes it to *max_entry (may be NULL). tau = 0 (the default) gives A_s^T. The
 * strip model needs det_spacing <= 1.4 (ABG_EINVAL otherwise). Not to be changed while a
 * solve uses the geometry. */
int abg_geometry_set_strip_threshold(abg_geometry *g, double tau, double *max_entry);

/* ---- operators -------------------------------------------------------------------- */

/* Device scratch (bytes) abg_fp_apply needs for dtype t: two zero-padded copies of the
 * image, one row-major and one transposed. */
size_t abg_fp_workspace_bytes(const abg_geometry *g, int dtype);

/* y = A x (the geometry's model, ray-driven). x: n elements, y: m elements, both of `dtype`
 * (ABG_F64 or ABG_F32); ws: abg_fp_workspace_bytes(g, dtype) bytes, 256-byte aligned.
 * Asynchronous on `stream`. */
int abg_fp_apply(const abg_geometry *g, int dtype, const void *x, void *y,
                 void *ws, size_t ws_bytes, void *stream);

/* y = A x like abg_fp_apply, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the two padded
 * copies of the image live in a static device array of the library (72 MiB per device,
 * held from the library's load until the process ends) instead of a caller workspace.
 * The call allocates nothing (no hipMalloc, no events, no library routine that
 * allocates); the caller still owns x and y. Limit: abg_fp_workspace_bytes(g, dtype) must
 * not exceed 72 MiB (N <= 2168 in FP64, N <= 3068 in FP32); larger geometries return
 * ABG_ENOMEM and launch nothing. Every call on a device shares that device's array and
 * clears what must start at zero itself; calls that overlap in time on one device (other
 * streams, other threads) race on the array and must not be issued. Asynchronous on
 * `stream`; results are bit-for-bit those of abg_fp_apply. */
int abg_fp_apply_noalloc(const abg_geometry *g, int dtype, const void *x, void *y, void *stream);

/* x = B y for kind ABG_BP_HAT (unmatched), x = A_line^T y for ABG_BP_ADJ, A_strip^T y for
 * ABG_BP_STRIP_T, A_Joseph^T y for ABG_BP_JOSEPH_T, B_tau y for ABG_BP_STRIP_TAU; pixel
 * driven. y: m elements, x: n elements of `dtype`. Asynchronous on `stream`. */
int abg_bp_apply(const abg_geometry *g, int kind, int dtype, const void *y, void *x,
                 void *stream);

/* ---- solvers (Sec. 2) ------------------------------------------------------------- */

/* Device workspace (bytes) of one AB (method 0) or BA (method 1) solve with k_max steps. */
size_t abg_workspace_bytes(const abg_geometry *g, int method, int k_max, abg_precision p,
                           abg_stop st);

/* AB-GMRES. b: m elements (p.proj), x0: n elements or NULL for x_0 = 0, x: n elements
 * (output; may not alias b or x0). ws: abg_workspace_bytes(...) bytes, 256-byte aligned.
 * info may be NULL. Returns ABG_OK, ABG_NOT_CONVERGED, ABG_BREAKDOWN, ABG_ZERO_RHS or an
 * error; on error x is unspecified. Synchronises `stream` before returning. */
int abg_ab_gmres(const abg_geometry *g, int bp_kind, const void *b, const void *x0, void *x,
                 int k_max, abg_stop st, abg_precision p, void *ws, size_t ws_bytes,
                 abg_info *info, void *stream);

/* BA-GMRES, same arguments. */
int abg_ba_gmres(const abg_geometry *g, int bp_kind, const void *b, const void *x0, void *x,
                 int k_max, abg_stop st, abg_precision p, void *ws, size_t ws_bytes,
                 abg_info *info, void *stream);

/* Error history of a finished solve (the semi-convergence curves of Sec. 6.2: the error
 * of each iterate against a known image falls, reaches a minimum, then grows as noise
 * is fitted). Called after abg_ab_gmres (method 0) or abg_ba_gmres (method 1) returned
 * on `ws` with the same g, bp_kind, k_max, st, p and x0, before ws is used again:
 * err[k-1] = ||x_k - x_ref||_2 for k = 1..k_done (host array of k_done doubles), where
 * x_k is rebuilt from the basis and the k-step small-problem solution that the solve
 * left in ws, so k_done may not exceed the steps the solve completed (info->k_done).
 * x_ref: n elements of p.proj (device). Overwrites the solve's scratch vectors (not x).
 * Synchronises `stream`. Returns ABG_EINVAL when ws holds fewer than k_done completed
 * steps or an argument is invalid. */
int abg_gmres_error_history(const abg_geometry *g, int method, int bp_kind, int k_max,
                            abg_stop st, abg_precision p, const void *x0, const void *x_ref,
                            void *ws, size_t ws_bytes, int k_done, double *err,
                            void *stream);

/* ---- matched comparators (Sec. 5, 6.2) ----------------------------------------------- */
/*
 * LSQR (Paige & Saunders) and LSMR (Fong & Saunders): the methods AB-GMRES and BA-GMRES
 * become with B = A^T (Sec. 5), run by the paper as comparators (Table 6.3). A is the
 * geometry's forward model and the back projector its exact transpose. Golub-Kahan
 * bidiagonalisation with short recurrences (no basis is stored; no reorthogonalisation),
 * FP64 scalars. LSQR minimises ||b - A x|| over K_k(A^T A, A^T r_0), LSMR ||A^T (b - A x)||.
 * Stopping rules ABG_STOP_NONE, ABG_STOP_DP (the residual estimate -- LSQR's phibar,
 * LSMR's recurred residual -- raises a candidate, confirmed with ||b - A x_k||) and
 * ABG_STOP_NCP (Sec. 6.3: every step forms the explicit residual b - A x_k, one extra
 * forward projection, and its periodogram distance d_k; the first k >= 2 with
 * d_k > d_{k-1} returns x_{k-1}, kept by the step; without such a k, x_{k_max}, the
 * iterate of smallest d). info->res_hist receives the residual estimates (explicit
 * residual norms in NCP runs), info->ls_hist the estimates of ||A^T r_k||, ncp_hist d_k
 * (NCP runs); info->H is not filled. Returns as abg_ab_gmres; ABG_BREAKDOWN when the
 * bidiagonalisation ends (alpha or beta = 0: x_k solves the least squares problem).
 * b: m elements, x0 (or NULL) and x: n elements, all of `dtype` (ABG_F64 or ABG_F32,
 * device); ws: abg_lsq_workspace_bytes(g, method, dtype) bytes, 256-byte aligned; k_max
 * in 1..500. Error history (Sec. 6.2): with x_ref (n elements of dtype, device) and
 * err_hist (host, k_max doubles) both given, err_hist[k-1] = ||x_k - x_ref||_2 for every
 * step performed; both NULL otherwise. Synchronises `stream` before returning.
 */
size_t abg_lsq_workspace_bytes(const abg_geometry *g, int method, int dtype);
int abg_lsqr(const abg_geometry *g, const void *b, const void *x0, void *x, int k_max,
             abg_stop st, int dtype, void *ws, size_t ws_bytes, abg_info *info,
             const void *x_ref, double *err_hist, void *stream);
int abg_lsmr(const abg_geometry *g, const void *b, const void *x0, void *x, int k_max,
             abg_stop st, int dtype, void *ws, size_t ws_bytes, abg_info *info,
             const void *x_ref, double *err_hist, void *stream);

/* Static description of a status code. */
const char *abg_status_string(int status);

/* ---- batched engine: many independent solves advanced together ---------------------- */
/*
 * An engine advances every problem it holds by one Arnoldi step per round (the same
 * AB-/BA-GMRES iteration as above: A, B, modified Gram-Schmidt, FP64 Givens, the DP
 * test), with all problems' work in one fixed sequence of kernels that is captured once
 * in a HIP graph and replayed. Problems of any geometry, method, back projector and
 * iteration cap share a round; each stops on its own rule, and a new problem can be
 * submitted between any two rounds (continuous batching). A problem's result does not
 * depend on which other problems share its rounds.
 *
 * Threading: one host thread per engine. All device work is enqueued on the engine's
 * stream. Stopping rules: ABG_STOP_NONE and ABG_STOP_DP (NCP is single-solve only);
 * info->H and info->ncp_hist are not filled.
 */
typedef struct abg_engine abg_engine;

typedef struct {
    const abg_geometry *g;   /* geometry on the engine's device; must outlive the request */
    int method;              /* ABG_METHOD_AB or ABG_METHOD_BA                             */
    int bp_kind;             /* ABG_BP_HAT or ABG_BP_ADJ (line-model geometries only)      */
    int k_max;               /* 1..500                                                     */
    abg_stop stop;           /* ABG_STOP_NONE or ABG_STOP_DP                               */
    const void *b;           /* m elements of the engine's proj dtype (device)             */
    const void *x0;          /* n elements, or NULL for x_0 = 0                            */
    void *x;                 /* n elements: the result (device)                            */
    void *ws;                /* abg_request_bytes(...) bytes, 256-byte aligned (device)    */
    size_t ws_bytes;
    abg_info *info;          /* host, may be NULL; filled when the request is finished      */
    long long tag;           /* caller's identifier, reported by abg_engine_poll          */
} abg_request;

/* Device memory one request needs (its Krylov basis, Hessenberg state and scratch): the
 * unit of admission against a memory budget. Same value as abg_workspace_bytes. */
size_t abg_request_bytes(const abg_geometry *g, int method, int k_max, abg_precision p,
                         abg_stop st);

/* Creates an engine on the current device for up to max_slots (1..4096) concurrent
 * problems. p: {F64,F64}, {F32,F32} or {F32,BF16}. The engine owns a few small device
 * and pinned host buffers (descriptors, work lists, scalar copies). */
int abg_engine_create(abg_precision p, int max_slots, void *stream, abg_engine **out);

/* Synchronises the stream and releases the engine; unfinished problems are abandoned. */
int abg_engine_destroy(abg_engine *e);

/* Adds a problem. Its buffers (b, x0, x, ws) belong to the engine until abg_engine_poll
 * has returned its tag. Enqueues the initialisation (r_0, beta, w_1) without waiting.
 * Returns ABG_EFULL when no slot is free, ABG_EINVAL on bad arguments (including a basis
 * vector too long for one block group, or a sinogram of 2 GiB or more in the projector
 * dtype: the engine's back projector addresses it with 31-bit offsets). */
int abg_engine_submit(abg_engine *e, const abg_request *r);

/* Runs one round: enqueues one Arnoldi step of every running problem and processes the
 * scalars of the previous round (at most one round is left in flight). Problems found
 * finished become available to abg_engine_poll. *n_active (may be NULL) receives the
 * number of problems not yet finished. */
int abg_engine_step(abg_engine *e, int *n_active);

/* Returns up to `max` finished problems (tags and statuses, in finishing order). After
 * this, their x holds the result and their buffers are the caller's again. */
int abg_engine_poll(abg_engine *e, long long *tags, int *status, int max, int *n);

/* Tile shapes and schedule of the projector work items, taking effect next round.
 * rays: rays of one angle per forward-projector block (64, 128 or 256; a block of 256
 * threads takes 256/rays angles), or 0 (the default): per problem, the shape single
 * solves of its geometry use (abg_fp_force_block_shape). ang_block: angles whose detector
 * windows a back-projector block stages in LDS per round (64, the default, or 128). sched:
 * 0 deals the items out round-robin over the resident blocks; 1 cuts each
 * item list into 8 contiguous ranges, one per XCD, that blocks drain through per-range
 * counters in shrinking chunks (half of what is left over the blocks of the range) before
 * helping with the others; 2 (the default) hands the whole list out in order through one
 * counter, in shrinking chunks, so that all blocks work on the same one or two problems
 * at a time.
 * Results do not depend on any of them. */
int abg_engine_set_tiles(abg_engine *e, int rays, int ang_block, int sched);
int abg_engine_get_tiles(const abg_engine *e, int *rays, int *ang_block, int *sched);

/* Autotuner: times the projector phases of one round for every tile shape and schedule
 * on the problems the engine holds (after `reps` repetitions each, without advancing
 * them), keeps the fastest and returns it with its time in ms. Synchronises the stream.
 * With no running problem it keeps the current choice and returns ms = 0. */
int abg_engine_autotune(abg_engine *e, int reps, int *rays, int *ang_block, int *sched,
                        double *ms);

/* Convenience: solves n requests together on a new engine and returns when all are
 * finished (each request's status in its info, if given). Returns the first error, or
 * ABG_OK. rays / ang_block <= 0 and sched < 0 keep the defaults. */
int abg_batch_solve(const abg_request *r, int n, abg_precision p, int rays, int ang_block,
                    int sched, void *stream);

/* ---- instrumentation -------------------------------------------------------------- */

/* When enabled, solver calls bracket every forward- and back-projector launch with HIP
 * events on the solver's stream and accumulate their durations (process-wide). Enabling
 * creates the events it will need (about 8k, on the current device); the durations are
 * read by abg_profile_read (or once 4096 launches are pending), so solves do not wait
 * for them. */
int abg_profile_enable(int on);
/* Reads and (if reset) clears the accumulated counts and milliseconds (arrays of
 * ABG_PROF_KINDS entries, caller-owned): index 0 forward projector, 1 back projector,
 * 2 Gram-Schmidt, 3 basis combination, 4 NCP evaluation (its three kernels). */
#define ABG_PROF_KINDS 5
int abg_profile_read(long long counts[ABG_PROF_KINDS], double ms[ABG_PROF_KINDS], int reset);

/* NCP periodograms (Sec. 6.3) take the DFT of every sinogram row by Bluestein's chirp
 * transform (two power-of-two FFTs in LDS; rows of 64 to 4096 bins), with tables of
 * at most 256 KB that the first NCP solve on a geometry builds on the host and keeps in
 * device memory until the geometry is destroyed; other row lengths use Goertzel's
 * recurrence per frequency. With on != 0 every row length uses the recurrence
 * (process-wide; for tests and measurements). Returns ABG_OK. */
int abg_ncp_force_goertzel(int on);

/* Block shape of the forward projectors (line, strip and Joseph models): each block of
 * 256 threads takes 2^lg_angles consecutive angles and 256 / 2^lg_angles consecutive rays
 * of each (0: one angle, 1: two, 2: four). -1 (the default) chooses by image size: four
 * angles for N > 512, else one, or two where that leaves fewer lanes of the last block of
 * each angle idle. The shape changes only
 * which rays run together, never a ray's arithmetic: results are bit-identical for every
 * shape. Process-wide; for tests and measurements. Returns ABG_OK, or ABG_EINVAL for
 * lg_angles outside -1..2. */
int abg_fp_force_block_shape(int lg_angles);

/* Share of the four-angle forward-projector blocks (line model) that stage each band
 * row's columns in LDS and read their taps there, in eighths (0..8), spread over the grid;
 * the other blocks read their taps from the image copies. The two kinds take their taps
 * through different units of a compute unit, so a mix of them gathers faster than either
 * alone. -1 (the default) restores the automatic share: three eighths in FP32; in FP64
 * two at N = 1024 and three below while N times the angle step (radians) is at most 4,
 * else none (the engine's forward items: FP32 three, FP64 none). Results are
 * bit-identical for every share. Process-wide; for tests and measurements. Returns ABG_OK, or ABG_EINVAL
 * for eighths outside -1..8. */
int abg_fp_force_stage_share(int eighths);

/* Releases what the library holds process-wide beyond geometries and engines: the
 * profiling events (profiling is switched off; accumulated counts are kept) and the idle
 * pooled pinned scalar slots and events of single solves (a solve leases one set for its
 * duration). Call it with no library call in flight on any thread, before the HIP
 * runtime shuts down (e.g. at the end of a program), so that nothing is left to static
 * destructors at process exit; later calls re-create what they need. Returns ABG_OK. */
int abg_release_process_resources(void);

/* Single solves whose basis vectors are longer than 2^21 elements carry an FP64 scratch
 * vector and switch to a streaming Gram-Schmidt variant (q_k in that scratch, one pass per
 * inner product) when q_k does not fit the registers of the blocks the device holds at
 * once. With on != 0 they always take the streaming variant (process-wide; for tests
 * and measurements). */
int abg_mgs_force_stream(int on);

#ifdef __cplusplus
}
#endif
#endif /* ABGMRES_H */
