/*
 * FP64 reference projectors for 2-D parallel-beam CT -- TEST INFRASTRUCTURE ONLY.
 *
 * Part of the reference oracle: only the test-suite, the smoke check and the CPU
 * baseline of the benchmark load this library. It shares no code with the GPU path.
 *
 * Conventions (the paper leaves them open; Sec. 6.1 and Table 6.1 fix only sizes):
 *   image  : N x N unit pixels centred on the origin; pixel (r, c), linear index
 *            j = r*N + c, covers [c-N/2, c-N/2+1] x [r-N/2, r-N/2+1].
 *   angles : omega_a = (cos th_a, sin th_a), passed in by the caller.
 *   rays   : line {p : <p, omega_a> = s_i}, s_i = (i - (n_det-1)/2) * ds,
 *            sinogram index a*n_det + i.
 *
 * A (line model, eq. 1.1's forward projector): A[(a,i), j] = length of ray (a,i)
 * inside pixel j. For a unit square whose centre projects to t0 on omega, this
 * length is a trapezoid in t = s - t0: with p = max(|cos|,|sin|), q = min(...),
 *     1/p                     for |t| <= (p-q)/2,
 *     ((p+q)/2 - |t|)/(p q)   for (p-q)/2 < |t| < (p+q)/2,
 *     0                       otherwise;
 * for q = 0 (axis-aligned rays) it is 1 for |t| < 1/2, 0 for |t| > 1/2 and 1/2 at
 * |t| = 1/2: a ray along a pixel edge is split evenly between the two pixels.
 *
 * B (unmatched back projector): B[j, (a,i)] = max(0, 1 - |u - i|) / ds with
 * u = (<c_j, omega_a> - s_0)/ds: linear interpolation of the sinogram row at the
 * detector position of the pixel centre, scaled so that B approximates A^T.
 *
 * Two further discretisation models of A (Sec. 6.1 names the line, strip and
 * interpolation (Joseph) models), with t = s_i - t0 as above:
 *
 * A_s (strip model): ray (a,i) is the strip of width ds centred on s_i, and the weight is
 * the area of strip and pixel divided by ds. By Cavalieri the area is the integral of
 * the line-model trapezoid over the strip, so
 *     A_s[(a,i), j] = (G(t + ds/2) - G(t - ds/2)) / ds,
 * G the antiderivative of the trapezoid (G(-inf) = 0, G(+inf) = 1: the pixel's area).
 *
 * A_i (Joseph's interpolation model): along the major axis of the ray (rows when
 * |cos| >= |sin|), the image row is interpolated linearly at the point where the ray
 * crosses the row's centre line, and the sample is weighted by the ray's length in the
 * row, 1/p. A pixel whose centre lies a distance d from that crossing point (in pixels
 * along the row) gets (1/p)(1 - d) for d < 1; since d = |t|/p, in detector coordinates
 *     A_i[(a,i), j] = max(0, 1 - |t|/p) / p,
 * a triangle of half-width p (pixels beyond the image edge count as zero).
 *
 * The operators are evaluated pixel-driven from these closed forms, with an explicit
 * loop over the detector bins each pixel can reach.
 */
#include <math.h>
#include <stddef.h>

/* An axis-aligned ray counts as lying on a pixel edge when its offset from the pixel
 * centre is within EDGE_TIE of 1/2: bin positions s0 + i*ds carry rounding error, and
 * a ray that lies on the edge in exact arithmetic must be recognised as such. */
#define EDGE_TIE 1e-9

static double trap(double t, double p, double q)
{
    double at = fabs(t);
    if (q == 0.0) {
        /* on a pixel edge (|t| = 1/2 up to rounding of the bin position) */
        if (fabs(at - 0.5) <= EDGE_TIE) return 0.5 / p;
        if (at < 0.5) return 1.0 / p;
        return 0.0;
    }
    double flat = 0.5 * (p - q), outer = 0.5 * (p + q);
    if (at <= flat) return 1.0 / p;
    if (at >= outer) return 0.0;
    return (outer - at) / (p * q);
}

/* Antiderivative of the trapezoid trap(., p, q) (unit area), from -inf to x. */
static double trap_int(double x, double p, double q)
{
    double a = fabs(x);
    double h0 = 0.5 * (p - q), h1 = 0.5 * (p + q);
    double below;   /* integral from -inf to -a */
    if (a >= h1)
        below = 0.0;
    else if (a >= h0)
        below = (h1 - a) * (h1 - a) / (2.0 * p * q);
    else
        below = (q > 0.0 ? 0.5 * q / p : 0.0) + (h0 - a) / p;
    return x < 0.0 ? below : 1.0 - below;
}

/* Weight of ray (a,i) at pixel j for model 0 (line), 1 (strip), 2 (Joseph); t = s_i - t0. */
static double model_w(int model, double t, double p, double q, double ds)
{
    if (model == 1) return (trap_int(t + 0.5 * ds, p, q) - trap_int(t - 0.5 * ds, p, q)) / ds;
    if (model == 2) {
        double a = 1.0 - fabs(t) / p;
        return a > 0.0 ? a / p : 0.0;
    }
    return trap(t, p, q);
}

/* Half-width (in t) of the support of model_w. */
static double model_reach(int model, double p, double q, double ds)
{
    if (model == 1) return 0.5 * (p + q) + 0.5 * ds;
    if (model == 2) return p;
    return 0.5 * (p + q);
}

static double hat(double v)
{
    double a = 1.0 - fabs(v);
    return a > 0.0 ? a : 0.0;
}

static void pixel_centre(int N, int j, double *xc, double *yc)
{
    int r = j / N, c = j % N;
    *xc = (double)c - 0.5 * N + 0.5;
    *yc = (double)r - 0.5 * N + 0.5;
}

/* Range of bins i whose centre s_i lies within `reach` of position t0. */
static void bin_range(double t0, double reach, double s0, double ds, int n_det,
                      int *i_lo, int *i_hi)
{
    int lo = (int)floor((t0 - reach - s0) / ds) - 1;
    int hi = (int)ceil((t0 + reach - s0) / ds) + 1;
    if (lo < 0) lo = 0;
    if (hi > n_det - 1) hi = n_det - 1;
    *i_lo = lo;
    *i_hi = hi;
}

/* y = A x. Each thread owns whole sinogram rows (one angle), so no two threads
 * write the same entry and the summation order is fixed. */
void orc_forward(int N, int n_ang, const double *cs, const double *sn, int n_det,
                 double ds, const double *x, double *y)
{
    const double s0 = -0.5 * (n_det - 1) * ds;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int a = 0; a < n_ang; ++a) {
        double c = cs[a], s = sn[a];
        double p = fmax(fabs(c), fabs(s)), q = fmin(fabs(c), fabs(s));
        double *row = y + (size_t)a * n_det;
        for (int i = 0; i < n_det; ++i) row[i] = 0.0;
        for (int j = 0; j < N * N; ++j) {
            if (x[j] == 0.0) continue;
            double xc, yc;
            pixel_centre(N, j, &xc, &yc);
            double t0 = xc * c + yc * s;
            int lo, hi;
            bin_range(t0, 0.5 * (p + q), s0, ds, n_det, &lo, &hi);
            for (int i = lo; i <= hi; ++i) {
                double si = s0 + i * ds;
                row[i] += trap(si - t0, p, q) * x[j];
            }
        }
    }
}

/* x = A^T y, one pixel per loop iteration. */
void orc_adjoint(int N, int n_ang, const double *cs, const double *sn, int n_det,
                 double ds, const double *y, double *x)
{
    const double s0 = -0.5 * (n_det - 1) * ds;
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < N * N; ++j) {
        double xc, yc, acc = 0.0;
        pixel_centre(N, j, &xc, &yc);
        for (int a = 0; a < n_ang; ++a) {
            double c = cs[a], s = sn[a];
            double p = fmax(fabs(c), fabs(s)), q = fmin(fabs(c), fabs(s));
            double t0 = xc * c + yc * s;
            int lo, hi;
            bin_range(t0, 0.5 * (p + q), s0, ds, n_det, &lo, &hi);
            for (int i = lo; i <= hi; ++i) {
                double si = s0 + i * ds;
                acc += trap(si - t0, p, q) * y[(size_t)a * n_det + i];
            }
        }
        x[j] = acc;
    }
}

/* x = B y with the pixel-driven linear-interpolation back projector. */
void orc_backproject_hat(int N, int n_ang, const double *cs, const double *sn, int n_det,
                         double ds, const double *y, double *x)
{
    const double s0 = -0.5 * (n_det - 1) * ds;
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < N * N; ++j) {
        double xc, yc, acc = 0.0;
        pixel_centre(N, j, &xc, &yc);
        for (int a = 0; a < n_ang; ++a) {
            double t0 = xc * cs[a] + yc * sn[a];
            double u = (t0 - s0) / ds;
            int lo, hi;
            bin_range(t0, ds, s0, ds, n_det, &lo, &hi);
            for (int i = lo; i <= hi; ++i)
                acc += hat(u - i) * y[(size_t)a * n_det + i];
        }
        x[j] = acc / ds;
    }
}

/* y = A_model x (model 0 line, 1 strip, 2 Joseph); rows owned by threads as above. */
void orc_forward_model(int model, int N, int n_ang, const double *cs, const double *sn,
                       int n_det, double ds, const double *x, double *y)
{
    const double s0 = -0.5 * (n_det - 1) * ds;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int a = 0; a < n_ang; ++a) {
        double c = cs[a], s = sn[a];
        double p = fmax(fabs(c), fabs(s)), q = fmin(fabs(c), fabs(s));
        double *row = y + (size_t)a * n_det;
        for (int i = 0; i < n_det; ++i) row[i] = 0.0;
        for (int j = 0; j < N * N; ++j) {
            if (x[j] == 0.0) continue;
            double xc, yc;
            pixel_centre(N, j, &xc, &yc);
            double t0 = xc * c + yc * s;
            int lo, hi;
            bin_range(t0, model_reach(model, p, q, ds), s0, ds, n_det, &lo, &hi);
            for (int i = lo; i <= hi; ++i)
                row[i] += model_w(model, s0 + i * ds - t0, p, q, ds) * x[j];
        }
    }
}

/* x = A_model^T y, one pixel per loop iteration. */
void orc_transpose_model(int model, int N, int n_ang, const double *cs, const double *sn,
                         int n_det, double ds, const double *y, double *x)
{
    const double s0 = -0.5 * (n_det - 1) * ds;
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < N * N; ++j) {
        double xc, yc, acc = 0.0;
        pixel_centre(N, j, &xc, &yc);
        for (int a = 0; a < n_ang; ++a) {
            double c = cs[a], s = sn[a];
            double p = fmax(fabs(c), fabs(s)), q = fmin(fabs(c), fabs(s));
            double t0 = xc * c + yc * s;
            int lo, hi;
            bin_range(t0, model_reach(model, p, q, ds), s0, ds, n_det, &lo, &hi);
            for (int i = lo; i <= hi; ++i)
                acc += model_w(model, s0 + i * ds - t0, p, q, ds) * y[(size_t)a * n_det + i];
        }
        x[j] = acc;
    }
}

/* Frobenius inner products <A_a, A_b>_F of the three models (3 x 3, row-major into G),
 * for the norm-wise model differences of Table 6.2. */
void orc_model_gram(int N, int n_ang, const double *cs, const double *sn, int n_det,
                    double ds, double *G)
{
    const double s0 = -0.5 * (n_det - 1) * ds;
    double acc[9] = {0};
    #pragma omp parallel
    {
        double loc[9] = {0};
        #pragma omp for schedule(static)
        for (int j = 0; j < N * N; ++j) {
            double xc, yc;
            pixel_centre(N, j, &xc, &yc);
            for (int a = 0; a < n_ang; ++a) {
                double c = cs[a], s = sn[a];
                double p = fmax(fabs(c), fabs(s)), q = fmin(fabs(c), fabs(s));
                double t0 = xc * c + yc * s;
                int lo, hi;
                bin_range(t0, model_reach(1, p, q, ds), s0, ds, n_det, &lo, &hi);
                for (int i = lo; i <= hi; ++i) {
                    double t = s0 + i * ds - t0, w[3];
                    for (int m = 0; m < 3; ++m) w[m] = model_w(m, t, p, q, ds);
                    for (int m = 0; m < 3; ++m)
                        for (int k = 0; k < 3; ++k) loc[3 * m + k] += w[m] * w[k];
                }
            }
        }
        #pragma omp critical
        for (int m = 0; m < 9; ++m) acc[m] += loc[m];
    }
    for (int m = 0; m < 9; ++m) G[m] = acc[m];
}

#define TAU_TIE 1e-6

/* Largest entry of the strip-model matrix (max over rays and pixels). */
double orc_strip_max(int N, int n_ang, const double *cs, const double *sn, int n_det, double ds)
{
    const double s0 = -0.5 * (n_det - 1) * ds;
    double best = 0.0;
    #pragma omp parallel for schedule(static) reduction(max : best)
    for (int j = 0; j < N * N; ++j) {
        double xc, yc;
        pixel_centre(N, j, &xc, &yc);
        for (int a = 0; a < n_ang; ++a) {
            double c = cs[a], s = sn[a];
            double p = fmax(fabs(c), fabs(s)), q = fmin(fabs(c), fabs(s));
            double t0 = xc * c + yc * s;
            int lo, hi;
            bin_range(t0, model_reach(1, p, q, ds), s0, ds, n_det, &lo, &hi);
            for (int i = lo; i <= hi; ++i) {
                double w = model_w(1, s0 + i * ds - t0, p, q, ds);
                if (w > best) best = w;
            }
        }
    }
    return best;
}

/* x = B_tau y: the strip-model transpose without its entries below thr (Sec. 6.5, eq. for
 * B_tau with thr = tau * max A_s). Entries within TAU_TIE * max of the threshold count as
 * on it and are kept: ties such as a strip covering half a pixel at 0 degrees (weight
 * exactly 1/2) must be decided the same way by implementations that round differently. */
void orc_transpose_strip_tau(int N, int n_ang, const double *cs, const double *sn, int n_det,
                             double ds, double thr, double max_entry, const double *y, double *x)
{
    const double s0 = -0.5 * (n_det - 1) * ds;
    const double tie = TAU_TIE * max_entry;
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < N * N; ++j) {
        double xc, yc, acc = 0.0;
        pixel_centre(N, j, &xc, &yc);
        for (int a = 0; a < n_ang; ++a) {
            double c = cs[a], s = sn[a];
            double p = fmax(fabs(c), fabs(s)), q = fmin(fabs(c), fabs(s));
            double t0 = xc * c + yc * s;
            int lo, hi;
            bin_range(t0, model_reach(1, p, q, ds), s0, ds, n_det, &lo, &hi);
            for (int i = lo; i <= hi; ++i) {
                double w = model_w(1, s0 + i * ds - t0, p, q, ds);
                if (w >= thr - tie) acc += w * y[(size_t)a * n_det + i];
            }
        }
        x[j] = acc;
    }
}

/* Sums of squares of the strip-model entries: all of them (out[0]) and those B_tau drops
 * (out[1]), so that ||B_tau - A_s^T||_F / ||A_s||_F = sqrt(out[1] / out[0]). */
void orc_strip_tau_sums(int N, int n_ang, const double *cs, const double *sn, int n_det,
                        double ds, double thr, double max_entry, double *out)
{
    const double s0 = -0.5 * (n_det - 1) * ds;
    const double tie = TAU_TIE * max_entry;
    double all = 0.0, low = 0.0;
    #pragma omp parallel for schedule(static) reduction(+ : all, low)
    for (int j = 0; j < N * N; ++j) {
        double xc, yc;
        pixel_centre(N, j, &xc, &yc);
        for (int a = 0; a < n_ang; ++a) {
            double c = cs[a], s = sn[a];
            double p = fmax(fabs(c), fabs(s)), q = fmin(fabs(c), fabs(s));
            double t0 = xc * c + yc * s;
            int lo, hi;
            bin_range(t0, model_reach(1, p, q, ds), s0, ds, n_det, &lo, &hi);
            for (int i = lo; i <= hi; ++i) {
                double w = model_w(1, s0 + i * ds - t0, p, q, ds);
                all += w * w;
                if (w < thr - tie) low += w * w;
            }
        }
    }
    out[0] = all;
    out[1] = low;
}

/* Number of threads OpenMP will use (reported with CPU timings). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
