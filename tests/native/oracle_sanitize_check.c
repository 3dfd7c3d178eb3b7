/* The oracle's C projectors (oracle/projectors.c, compiled into this driver) under the
 * address and undefined-behaviour sanitizers: every entry point on small geometries with
 * ragged sizes, axis-aligned angles, several detector spacings and a limited angular
 * range; the matched pairs must satisfy the adjoint identity and every output must be
 * finite. Built and run by tests/test_sanitizers_host.py; prints "ok" on success. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "projectors.c"

static int failures = 0;
#define CHECK(c, ...)                                        \
    do {                                                     \
        if (!(c)) {                                          \
            printf("FAILED: " __VA_ARGS__);                  \
            printf("\n");                                    \
            ++failures;                                      \
        }                                                    \
    } while (0)

static double urand(unsigned long long *s)
{
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*s >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

static double dot(const double *a, const double *b, size_t n)
{
    double s = 0.0;
    for (size_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static int finite_all(const double *a, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

static void run(int N, int n_ang, int n_det, double range, double ds, unsigned long long seed)
{
    const size_t n = (size_t)N * N, m = (size_t)n_ang * n_det;
    double *cs = malloc(sizeof(double) * n_ang), *sn = malloc(sizeof(double) * n_ang);
    for (int a = 0; a < n_ang; ++a) {
        const double th = a * range / n_ang;
        const double r = th * 3.14159265358979323846 / 180.0;
        cs[a] = cos(r);
        sn[a] = sin(r);
        if (fmod(th, 90.0) == 0.0) {
            const long q = lround(th / 90.0) % 4;
            cs[a] = q == 0 ? 1.0 : q == 2 ? -1.0 : 0.0;
            sn[a] = q == 1 ? 1.0 : q == 3 ? -1.0 : 0.0;
        }
    }
    double *x = malloc(sizeof(double) * n), *y = malloc(sizeof(double) * m);
    double *Ax = malloc(sizeof(double) * m), *ATy = malloc(sizeof(double) * n);
    double *Bx = malloc(sizeof(double) * n);
    for (size_t i = 0; i < n; ++i) x[i] = urand(&seed);
    for (size_t i = 0; i < m; ++i) y[i] = urand(&seed);
    orc_forward(N, n_ang, cs, sn, n_det, ds, x, Ax);
    orc_adjoint(N, n_ang, cs, sn, n_det, ds, y, ATy);
    orc_backproject_hat(N, n_ang, cs, sn, n_det, ds, y, Bx);
    const double l = dot(Ax, y, m), r = dot(x, ATy, n);
    CHECK(fabs(l - r) <= 1e-11 * (fabs(l) + 1.0), "line adjoint N=%d n_ang=%d n_det=%d ds=%g: %g vs %g",
          N, n_ang, n_det, ds, l, r);
    CHECK(finite_all(Ax, m) && finite_all(ATy, n) && finite_all(Bx, n), "finite line/hat N=%d", N);
    for (int model = 0; model < 3; ++model) {
        if (model == 1 && ds > 1.4) continue;
        orc_forward_model(model, N, n_ang, cs, sn, n_det, ds, x, Ax);
        orc_transpose_model(model, N, n_ang, cs, sn, n_det, ds, y, ATy);
        const double l2 = dot(Ax, y, m), r2 = dot(x, ATy, n);
        CHECK(fabs(l2 - r2) <= 1e-11 * (fabs(l2) + 1.0), "model %d adjoint N=%d n_det=%d ds=%g: %g vs %g",
              model, N, n_det, ds, l2, r2);
    }
    double G[9];
    orc_model_gram(N, n_ang, cs, sn, n_det, ds, G);
    CHECK(finite_all(G, 9), "gram N=%d", N);
    if (ds <= 1.4) {
        const double mx = orc_strip_max(N, n_ang, cs, sn, n_det, ds);
        CHECK(isfinite(mx) && mx >= 0.0, "strip max N=%d", N);
        double sums[2];
        orc_transpose_strip_tau(N, n_ang, cs, sn, n_det, ds, 0.3 * mx, mx, y, ATy);
        orc_strip_tau_sums(N, n_ang, cs, sn, n_det, ds, 0.3 * mx, mx, sums);
        CHECK(finite_all(ATy, n) && sums[1] <= sums[0] + 1e-12, "strip tau N=%d", N);
    }
    free(cs); free(sn); free(x); free(y); free(Ax); free(ATy); free(Bx);
}

int main(void)
{
    const int Ns[] = {1, 2, 5, 16, 33};
    const int angs[] = {1, 4, 7, 24};
    const double dss[] = {0.75, 1.0, 1.3, 2.0};
    unsigned long long seed = 12345;
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 4; ++b)
            for (int c = 0; c < 4; ++c) {
                const int N = Ns[a];
                const int n_det = (int)ceil(N * 1.4143 / dss[c]) + 1 + (b % 2);
                run(N, angs[b], n_det, b == 3 ? 120.0 : 180.0, dss[c], seed++);
            }
    if (failures) return 1;
    printf("ok\n");
    return 0;
}
