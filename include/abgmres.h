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
 * the discrepancy principle or the NCP criterion (Sec. 6.3).
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
 *     output buffers.
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
#define ABG_NOT_CONVERGED 1    /* DP never satisfied up to k_max: x_{k_max} returned     */
#define ABG_BREAKDOWN 2        /* h_{k+1,k} ~ 0: Krylov space exhausted, x_k returned    */
#define ABG_ZERO_RHS 3         /* ||r_0|| = 0: x = x_0 returned with k = 0               */

typedef enum { ABG_F64 = 0, ABG_F32 = 1, ABG_BF16 = 2 } abg_dtype;
typedef enum { ABG_BP_HAT = 0, ABG_BP_ADJ = 1 } abg_bp_kind;
typedef enum { ABG_STOP_NONE = 0, ABG_STOP_DP = 1, ABG_STOP_NCP = 2 } abg_stop_kind;
typedef enum { ABG_METHOD_AB = 0, ABG_METHOD_BA = 1 } abg_method;

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
    double res_norm;     /* ||b - A x||_2 of the returned x, evaluated explicitly           */
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

/* ---- operators -------------------------------------------------------------------- */

/* Device scratch (bytes) abg_fp_apply needs for dtype t: two zero-padded copies of the
 * image, one row-major and one transposed. */
size_t abg_fp_workspace_bytes(const abg_geometry *g, int dtype);

/* y = A x (line model, ray-driven). x: n elements, y: m elements, both of `dtype`
 * (ABG_F64 or ABG_F32); ws: abg_fp_workspace_bytes(g, dtype) bytes, 256-byte aligned.
 * Asynchronous on `stream`. */
int abg_fp_apply(const abg_geometry *g, int dtype, const void *x, void *y,
                 void *ws, size_t ws_bytes, void *stream);

/* x = B y for kind ABG_BP_HAT (unmatched) or x = A^T y for ABG_BP_ADJ (matched), pixel
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

/* Static description of a status code. */
const char *abg_status_string(int status);

/* ---- instrumentation -------------------------------------------------------------- */

/* When enabled, solver calls bracket every forward- and back-projector launch with HIP
 * events on the solver's stream and accumulate their durations (process-wide). */
int abg_profile_enable(int on);
/* Reads and (if reset) clears the accumulated counts and milliseconds: index 0 forward
 * projector, 1 back projector, 2 Gram-Schmidt, 3 basis combination. */
int abg_profile_read(long long counts[4], double ms[4], int reset);

#ifdef __cplusplus
}
#endif
#endif /* ABGMRES_H */
