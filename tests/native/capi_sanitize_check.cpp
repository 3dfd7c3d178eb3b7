// The library's host code under AddressSanitizer and UBSan (_build/hostsan, built by
// paper_2110_01481_amd/build.py build_host_sanitized): this instrumented program calls
// every C-ABI entry point with invalid arguments (each must be refused before any device
// work) and, where a GPU is present, runs small solves of every kind: AB/BA-GMRES under
// each stop rule and precision, the error history, LSQR/LSMR, an engine with continuous
// admission, the projectors and the allocation-free forward projection, then releases
// everything. Prints "ok" when every check holds (the sanitizers abort on a finding).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "abgmres.h"

static int failures = 0;
#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            std::printf("FAILED: %s (line %d)\n", #c, __LINE__);  \
            ++failures;                                            \
        }                                                          \
    } while (0)

static void invalid_arguments()
{
    abg_geometry *g = nullptr;
    CHECK(abg_create_geometry(0, 10, 0, 180, nullptr, 11, 1.0, &g) == ABG_EINVAL);
    CHECK(abg_create_geometry(16, 0, 0, 180, nullptr, 11, 1.0, &g) == ABG_EINVAL);
    CHECK(abg_create_geometry(16, 10, 0, 180, nullptr, 0, 1.0, &g) == ABG_EINVAL);
    CHECK(abg_create_geometry(16, 10, 0, 180, nullptr, 11, 0.5, &g) == ABG_EINVAL);
    CHECK(abg_create_geometry(16, 10, 0, NAN, nullptr, 11, 1.0, &g) == ABG_EINVAL);
    CHECK(abg_create_geometry(16, 10, 0, 180, nullptr, 11, 1.0, nullptr) == ABG_EINVAL);
    const double bad_angles[3] = {0.0, NAN, 10.0};
    CHECK(abg_create_geometry(16, 3, 0, 0, bad_angles, 11, 1.0, &g) == ABG_EINVAL);
    CHECK(abg_destroy_geometry(nullptr) == ABG_OK);
    long long n = 0, m = 0;
    CHECK(abg_geometry_sizes(nullptr, &n, &m) != ABG_OK);
    CHECK(abg_fp_workspace_bytes(nullptr, ABG_F32) == 0);
    CHECK(abg_fp_apply(nullptr, ABG_F32, nullptr, nullptr, nullptr, 0, nullptr) == ABG_EINVAL);
    CHECK(abg_fp_apply_noalloc(nullptr, ABG_F32, nullptr, nullptr, nullptr) == ABG_EINVAL);
    CHECK(abg_bp_apply(nullptr, ABG_BP_HAT, ABG_F32, nullptr, nullptr, nullptr) == ABG_EINVAL);
    abg_stop st{ABG_STOP_NONE, 1.0, 0.0};
    abg_precision p{ABG_F32, ABG_F32};
    CHECK(abg_workspace_bytes(nullptr, 0, 10, p, st) == 0);
    CHECK(abg_request_bytes(nullptr, 0, 10, p, st) == 0);
    CHECK(abg_lsq_workspace_bytes(nullptr, ABG_METHOD_LSQR, ABG_F32) == 0);
    CHECK(abg_ab_gmres(nullptr, 0, nullptr, nullptr, nullptr, 10, st, p, nullptr, 0, nullptr, nullptr) ==
          ABG_EINVAL);
    CHECK(abg_ba_gmres(nullptr, 0, nullptr, nullptr, nullptr, 10, st, p, nullptr, 0, nullptr, nullptr) ==
          ABG_EINVAL);
    CHECK(abg_lsqr(nullptr, nullptr, nullptr, nullptr, 10, st, ABG_F32, nullptr, 0, nullptr, nullptr,
                   nullptr, nullptr) == ABG_EINVAL);
    CHECK(abg_lsmr(nullptr, nullptr, nullptr, nullptr, 10, st, ABG_F32, nullptr, 0, nullptr, nullptr,
                   nullptr, nullptr) == ABG_EINVAL);
    double err[4];
    CHECK(abg_gmres_error_history(nullptr, 0, 0, 10, st, p, nullptr, nullptr, nullptr, 0, 1, err,
                                  nullptr) == ABG_EINVAL);
    abg_engine *e = nullptr;
    abg_precision bad{ABG_F64, ABG_F32};
    CHECK(abg_engine_create(bad, 4, nullptr, &e) == ABG_EINVAL);
    CHECK(abg_engine_create(p, 0, nullptr, &e) == ABG_EINVAL);
    CHECK(abg_engine_destroy(nullptr) == ABG_OK || abg_engine_destroy(nullptr) == ABG_EINVAL);
    CHECK(abg_engine_submit(nullptr, nullptr) == ABG_EINVAL);
    CHECK(abg_engine_step(nullptr, nullptr) == ABG_EINVAL);
    CHECK(abg_geometry_set_model(nullptr, ABG_FP_STRIP) == ABG_EINVAL);
    CHECK(abg_geometry_set_strip_threshold(nullptr, 0.1, nullptr) == ABG_EINVAL);
    for (int code = -6; code <= 3; ++code) CHECK(abg_status_string(code) != nullptr);
    CHECK(std::strcmp(abg_status_string(99), "unknown status") == 0);
    CHECK(abg_mgs_force_stream(0) == ABG_OK);
    CHECK(abg_ncp_force_goertzel(0) == ABG_OK);
    long long counts[ABG_PROF_KINDS];
    double ms[ABG_PROF_KINDS];
    CHECK(abg_profile_read(counts, ms, 1) == ABG_OK);
    CHECK(abg_release_process_resources() == ABG_OK);
}

template <typename T> static T *dev(size_t n)
{
    void *p = nullptr;
    if (hipMalloc(&p, n * sizeof(T) + 256) != hipSuccess) return nullptr;
    return static_cast<T *>(p);
}

static void on_device()
{
    const int N = 48, n_ang = 60, n_det = 69;
    abg_geometry *g = nullptr;
    CHECK(abg_create_geometry(N, n_ang, 0, 180, nullptr, n_det, 1.0, &g) == ABG_OK);
    if (!g) return;
    const size_t n = (size_t)N * N, m = (size_t)n_ang * n_det;
    std::vector<double> hx(n);
    for (size_t j = 0; j < n; ++j) hx[j] = std::fabs(std::sin(0.37 * j)) * ((j / N) % 7 != 0);
    double *x = dev<double>(n), *b = dev<double>(m), *out = dev<double>(n), *xr = dev<double>(n);
    float *x32 = dev<float>(n), *b32 = dev<float>(m), *out32 = dev<float>(n);
    CHECK(x && b && out && xr && x32 && b32 && out32);
    hipMemcpy(x, hx.data(), n * 8, hipMemcpyHostToDevice);
    hipMemcpy(xr, hx.data(), n * 8, hipMemcpyHostToDevice);
    std::vector<float> hx32(hx.begin(), hx.end());
    hipMemcpy(x32, hx32.data(), n * 4, hipMemcpyHostToDevice);
    size_t fws = abg_fp_workspace_bytes(g, ABG_F64);
    void *ws = nullptr;
    hipMalloc(&ws, fws);
    CHECK(abg_fp_apply(g, ABG_F64, x, b, ws, fws, nullptr) == ABG_OK);
    CHECK(abg_fp_apply(g, ABG_F64, x, b, ws, fws - 1, nullptr) == ABG_ENOMEM);
    CHECK(abg_fp_apply_noalloc(g, ABG_F32, x32, b32, nullptr) == ABG_OK);
    for (int k = 0; k <= ABG_BP_STRIP_TAU; ++k) {
        if (k == ABG_BP_STRIP_TAU) CHECK(abg_geometry_set_strip_threshold(g, 0.2, nullptr) == ABG_OK);
        CHECK(abg_bp_apply(g, k, ABG_F64, b, out, nullptr) == ABG_OK);
    }
    hipFree(ws);
    hipDeviceSynchronize();
    std::vector<double> hb(m);
    hipMemcpy(hb.data(), b, m * 8, hipMemcpyDeviceToHost);
    double bn = 0.0;
    for (double v : hb) bn += v * v;
    const double enorm = 0.01 * std::sqrt(bn);
    std::vector<double> res(80), ls(80), ncp(80), H(81 * 80);
    for (int method = 0; method < 2; ++method)
        for (int stop = 0; stop < 3; ++stop)
            for (int prec = 0; prec < 3; ++prec) {
                abg_precision p = prec == 0 ? abg_precision{ABG_F64, ABG_F64}
                                  : prec == 1 ? abg_precision{ABG_F32, ABG_F32}
                                              : abg_precision{ABG_F32, ABG_BF16};
                abg_stop st{stop, 1.02, enorm};
                const int k_max = stop == ABG_STOP_NONE ? 70 : 40;
                size_t nb = abg_workspace_bytes(g, method, k_max, p, st);
                CHECK(nb > 0);
                void *w = nullptr;
                hipMalloc(&w, nb);
                abg_info info{};
                info.res_hist = res.data();
                info.ls_hist = ls.data();
                info.ncp_hist = ncp.data();
                info.hist_len = 80;
                info.H = prec == 0 ? H.data() : nullptr;
                const void *bb = prec == 0 ? (const void *)b : (const void *)b32;
                void *xo = prec == 0 ? (void *)out : (void *)out32;
                auto fn = method == 0 ? abg_ab_gmres : abg_ba_gmres;
                int rc = fn(g, ABG_BP_HAT, bb, nullptr, xo, k_max, st, p, w, nb, &info, nullptr);
                CHECK(rc >= 0);
                CHECK(fn(g, ABG_BP_HAT, bb, nullptr, xo, k_max, st, p, w, nb - 1, &info, nullptr) ==
                      ABG_ENOMEM);
                if (rc >= 0 && prec == 0 && info.k_done > 0) {
                    std::vector<double> eh(info.k_done);
                    CHECK(abg_gmres_error_history(g, method, ABG_BP_HAT, k_max, st, p, nullptr, xr,
                                                  w, nb, info.k_done, eh.data(), nullptr) == ABG_OK);
                }
                hipFree(w);
            }
    for (int method = ABG_METHOD_LSQR; method <= ABG_METHOD_LSMR; ++method) {
        size_t nb = abg_lsq_workspace_bytes(g, method, ABG_F64);
        void *w = nullptr;
        hipMalloc(&w, nb);
        abg_stop st{ABG_STOP_NCP, 1.0, 0.0};
        abg_info info{};
        std::vector<double> eh(30);
        auto fn = method == ABG_METHOD_LSQR ? abg_lsqr : abg_lsmr;
        CHECK(fn(g, b, nullptr, out, 30, st, ABG_F64, w, nb, &info, xr, eh.data(), nullptr) >= 0);
        hipFree(w);
    }
    // engine: six problems through three slots (continuous admission)
    abg_engine *e = nullptr;
    abg_precision p{ABG_F32, ABG_F32};
    CHECK(abg_engine_create(p, 3, nullptr, &e) == ABG_OK);
    if (e) {
        abg_stop st{ABG_STOP_DP, 1.02, enorm};
        std::vector<void *> wss(6), xs(6);
        std::vector<abg_info> infos(6);
        int submitted = 0, done = 0;
        long long tags[8];
        int status[8];
        for (int round = 0; round < 2000 && done < 6; ++round) {
            while (submitted < 6) {
                // each request's own method sizes its workspace
                const size_t nb = abg_request_bytes(g, submitted % 2, 40, p, st);
                hipMalloc(&wss[submitted], nb);
                hipMalloc(&xs[submitted], n * 4);
                abg_request r{g, submitted % 2, ABG_BP_HAT, 40, st, b32, nullptr, xs[submitted],
                              wss[submitted], nb, &infos[submitted], submitted};
                const int rc = abg_engine_submit(e, &r);
                if (rc == ABG_EFULL) {
                    hipFree(wss[submitted]);
                    hipFree(xs[submitted]);
                    break;
                }
                if (rc != ABG_OK) std::printf("engine submit %d: rc %d\n", submitted, rc);
                CHECK(rc == ABG_OK);
                ++submitted;
            }
            int active = 0;
            CHECK(abg_engine_step(e, &active) == ABG_OK);
            int got = 0;
            CHECK(abg_engine_poll(e, tags, status, 8, &got) == ABG_OK);
            done += got;
        }
        CHECK(done == 6);
        int rays = 0, ab = 0, sc = 0;
        CHECK(abg_engine_get_tiles(e, &rays, &ab, &sc) == ABG_OK);
        CHECK(abg_engine_set_tiles(e, 64, 64, 1) == ABG_OK);
        CHECK(abg_engine_set_tiles(e, 100, 64, 1) == ABG_EINVAL);
        CHECK(abg_engine_destroy(e) == ABG_OK);
        for (int i = 0; i < submitted; ++i) {
            hipFree(wss[i]);
            hipFree(xs[i]);
        }
    }
    CHECK(abg_profile_enable(1) == ABG_OK);
    {
        abg_stop st{ABG_STOP_NONE, 1.0, 0.0};
        abg_precision pp{ABG_F64, ABG_F64};
        size_t nb = abg_workspace_bytes(g, 1, 5, pp, st);
        void *w = nullptr;
        hipMalloc(&w, nb);
        CHECK(abg_ba_gmres(g, ABG_BP_HAT, b, nullptr, out, 5, st, pp, w, nb, nullptr, nullptr) == ABG_OK);
        hipFree(w);
    }
    long long counts[ABG_PROF_KINDS];
    double ms[ABG_PROF_KINDS];
    CHECK(abg_profile_read(counts, ms, 1) == ABG_OK && counts[0] > 0);
    CHECK(abg_profile_enable(0) == ABG_OK);
    hipFree(x); hipFree(b); hipFree(out); hipFree(xr); hipFree(x32); hipFree(b32); hipFree(out32);
    CHECK(abg_destroy_geometry(g) == ABG_OK);
    CHECK(abg_release_process_resources() == ABG_OK);
}

int main()
{
    invalid_arguments();
    int count = 0;
    if (hipGetDeviceCount(&count) == hipSuccess && count > 0) on_device();
    else std::printf("no GPU: argument checks only\n");
    // Everything this library holds has been released above. The process then ends
    // without its exit-time destructors: under the ROCm AddressSanitizer runtime, the HIP
    // runtime's own teardown after main returns frees host objects whose quarantine
    // recycling reaches device-memory chunks after the device runtime has been unloaded,
    // and the sanitizer stops on an internal CHECK there (code outside this library).
    std::printf(failures ? "failed\n" : "ok\n");
    std::fflush(stdout);
    std::_Exit(failures ? 1 : 0);
}
