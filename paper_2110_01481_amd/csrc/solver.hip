// AB-GMRES and BA-GMRES drivers (Sec. 2) with discrepancy-principle and NCP stopping
// (Sec. 6.3). The host thread only sequences kernels and reads back a few scalars per
// Arnoldi step; every vector operation runs in the kernels of this library.
//
// Per step k (BA):  z = A w_k (kept as column k of Z when a stopping rule needs the
// residual), q = B z, MGS, Givens, then r_k = (b - A x_0) - Z y_k.
// Per step k (AB):  t = B w_k, q = A t, MGS, Givens, then r_k = W_{k+1}(||r_0|| e_1 - H_k y_k).
// Both residual forms equal b - A x_k by linearity and the Arnoldi relation; the
// discrepancy principle confirms a candidate stop with the explicit b - A x_k.
#include <cmath>
#include <cstring>

#include "abg_internal.h"

namespace abg {
namespace {

struct Layout {
    size_t V, Z, cur, q, rb0, tm, tn, fpws, H, R, cs, sn, g, y, yprev, ybest, rho;
    size_t part, mgs_part, bar, st, ncp, total;
    long long L, ldv, mp, np;
};

long long round_up(long long v, long long a) { return (v + a - 1) / a * a; }

Layout make_layout(const Geometry &g, int method, int k_max, abg_precision p, abg_stop st)
{
    Layout ly{};
    const size_t sX = dtype_size(p.proj), sV = dtype_size(p.basis);
    ly.mp = round_up(g.m(), 128);
    ly.np = round_up(g.n(), 128);
    ly.L = method == ABG_METHOD_AB ? g.m() : g.n();
    ly.ldv = method == ABG_METHOD_AB ? ly.mp : ly.np;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    const bool need_res = st.kind != ABG_STOP_NONE;
    const size_t ld = (size_t)k_max + 1;
    ly.V = take(ld * ly.ldv * sV);
    ly.Z = (method == ABG_METHOD_BA && need_res) ? take((size_t)k_max * ly.mp * sX) : 0;
    ly.cur = take(ly.ldv * sX);
    ly.q = take(ly.ldv * sX);
    ly.rb0 = take(ly.mp * sX);
    ly.tm = take(ly.mp * sX);
    ly.tn = take(ly.np * sX);
    ly.fpws = take(fp_workspace_bytes(g, p.proj));
    ly.H = take(ld * k_max * 8);
    ly.R = take(ld * k_max * 8);
    ly.cs = take((size_t)k_max * 8);
    ly.sn = take((size_t)k_max * 8);
    ly.g = take(ld * 8);
    ly.y = take(ld * 8);
    ly.yprev = take(ld * 8);
    ly.ybest = take(ld * 8);
    ly.rho = take((ld + 1) * 8);
    ly.part = take(2048 * 8);
    ly.mgs_part = take(4 * (size_t)kMaxGrid * 8);
    ly.bar = take((ld + 2) * 4);
    ly.st = take(sizeof(DevState));
    ly.ncp = st.kind == ABG_STOP_NCP ? take(ncp_scratch_bytes(g)) : 0;
    ly.total = off;
    return ly;
}

struct HostState {
    DevState *h = nullptr;
    ~HostState()
    {
        if (h) (void)hipHostFree(h);
    }
};

#define CK(expr)                                   \
    do {                                           \
        hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) return ABG_EHIP;     \
    } while (0)

struct Solve {
    const Geometry &g;
    int method, kind, k_max;
    abg_stop st;
    abg_precision p;
    hipStream_t s;
    Layout ly;
    char *W;
    // views
    void *V, *Z, *cur, *q, *rb0, *tm, *tn, *fpws;
    double *H, *R, *cs, *sn, *gv, *y, *yprev, *ybest, *rho, *part, *mgs_part;
    unsigned *bar;
    DevState *dst;
    double *ncp;
    HostState hs;
    size_t sX;

    Solve(const Geometry &g_, int method_, int kind_, int k_max_, abg_stop st_,
          abg_precision p_, hipStream_t s_, void *ws)
        : g(g_), method(method_), kind(kind_), k_max(k_max_), st(st_), p(p_), s(s_)
    {
        ly = make_layout(g, method, k_max, p, st);
        W = static_cast<char *>(ws);
        V = W + ly.V;
        Z = ly.Z ? W + ly.Z : nullptr;
        cur = W + ly.cur;
        q = W + ly.q;
        rb0 = W + ly.rb0;
        tm = W + ly.tm;
        tn = W + ly.tn;
        fpws = W + ly.fpws;
        H = reinterpret_cast<double *>(W + ly.H);
        R = reinterpret_cast<double *>(W + ly.R);
        cs = reinterpret_cast<double *>(W + ly.cs);
        sn = reinterpret_cast<double *>(W + ly.sn);
        gv = reinterpret_cast<double *>(W + ly.g);
        y = reinterpret_cast<double *>(W + ly.y);
        yprev = reinterpret_cast<double *>(W + ly.yprev);
        ybest = reinterpret_cast<double *>(W + ly.ybest);
        rho = reinterpret_cast<double *>(W + ly.rho);
        part = reinterpret_cast<double *>(W + ly.part);
        mgs_part = reinterpret_cast<double *>(W + ly.mgs_part);
        bar = reinterpret_cast<unsigned *>(W + ly.bar);
        dst = reinterpret_cast<DevState *>(W + ly.st);
        ncp = ly.ncp ? reinterpret_cast<double *>(W + ly.ncp) : nullptr;
        sX = dtype_size(p.proj);
    }

    char *vec(int i) const { return static_cast<char *>(V) + (size_t)i * ly.ldv * dtype_size(p.basis); }
    char *zcol(int i) const { return static_cast<char *>(Z) + (size_t)i * ly.mp * sX; }

    int sync_state(DevState &out)
    {
        CK(hipMemcpyAsync(hs.h, dst, sizeof(DevState), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        out = *hs.h;
        return ABG_OK;
    }

    int fwd(const void *x, void *yv) { CK(launch_forward(g, p.proj, x, yv, fpws, s)); return ABG_OK; }
    int back(const void *yv, void *x) { CK(launch_back(g, kind, p.proj, yv, x, s)); return ABG_OK; }

    // norm of (a - b) into dst->res; result vector in out
    int sub_norm(const void *a, const void *b, void *out, long long L)
    {
        int nb = 0;
        CK(launch_sub_norm(p.proj, a, b, out, L, part, &nb, s));
        CK(launch_reduce_sqrt(part, nb, &dst->res, s));
        return ABG_OK;
    }

    // x = x0 + (BA) W[0..kk) c   or   x = x0 + B (W[0..kk) c)  (AB)
    int build_x(const double *c, int kk, const void *x0, void *x)
    {
        if (method == ABG_METHOD_BA) {
            CK(launch_combine(p.proj, x0, x0 ? 1.0 : 0.0, p.basis, V, ly.ldv, kk, c, 1.0, x,
                              g.n(), nullptr, nullptr, nullptr, s));
        } else {
            CK(launch_combine(p.proj, nullptr, 0.0, p.basis, V, ly.ldv, kk, c, 1.0, tm, g.m(),
                              nullptr, nullptr, nullptr, s));
            int rc = back(tm, x);
            if (rc) return rc;
            if (x0) CK(launch_axpy_inplace(p.proj, x, x0, g.n(), s));
        }
        return ABG_OK;
    }

    // explicit ||b - A x|| into dst->res (uses tm)
    int literal_residual(const void *b, const void *x)
    {
        int rc = fwd(x, tm);
        if (rc) return rc;
        return sub_norm(b, tm, tm, g.m());
    }
};

double dp_slack(int basis)
{
    return basis == ABG_F64 ? 1e-6 : (basis == ABG_F32 ? 1e-3 : 5e-2);
}

}  // namespace

size_t solver_workspace_bytes(const Geometry &g, int method, int k_max, abg_precision p,
                              abg_stop st)
{
    return make_layout(g, method, k_max, p, st).total;
}

int run_solver(const Geometry &g, int method, int kind, const void *b, const void *x0,
               void *x, int k_max, abg_stop st, abg_precision p, void *ws, size_t ws_bytes,
               abg_info *info, hipStream_t s)
{
    Solve S(g, method, kind, k_max, st, p, s, ws);
    if (ws_bytes < S.ly.total) return ABG_ENOMEM;
    CK(hipHostMalloc((void **)&S.hs.h, sizeof(DevState), hipHostMallocDefault));
    const long long m = g.m(), n = g.n(), L = S.ly.L;
    const int ld = k_max + 1;
    const bool need_res = st.kind != ABG_STOP_NONE;
    const double thr = st.kind == ABG_STOP_DP ? st.tau * st.noise_norm : 0.0;
    const double bd_rel = p.basis == ABG_F64 && p.proj == ABG_F64 ? 1e-14 : 1e-6;
    int k_stop = 0, k_done = 0, status = ABG_OK, n_literal = 0;
    double res_final = 0.0, ncp_final = 0.0;
    auto hist = [&](double *arr, int k, double v) {
        if (info && arr && k - 1 < info->hist_len) arr[k - 1] = v;
    };

    // small state to zero
    CK(launch_fill_u32(S.bar, (size_t)ld + 2, 0u, s));
    CK(launch_fill_u32(reinterpret_cast<unsigned *>(S.dst), sizeof(DevState) / 4, 0u, s));
    CK(launch_fill_f64(S.H, (size_t)ld * k_max, 0.0, s));
    CK(launch_fill_f64(S.gv, (size_t)ld, 0.0, s));

    // b - A x0, r0, beta, w1
    int rc;
    if (x0) {
        if ((rc = S.fwd(x0, S.tm))) return rc;
        if ((rc = S.sub_norm(b, S.tm, S.rb0, m))) return rc;
    } else {
        CK(hipMemcpyAsync(S.rb0, b, (size_t)m * S.sX, hipMemcpyDeviceToDevice, s));
    }
    const void *r0 = S.rb0;
    if (method == ABG_METHOD_BA) {
        if ((rc = S.back(S.rb0, S.q))) return rc;
        r0 = S.q;
    }
    MgsLaunch M{};
    M.tx = p.proj;
    M.tv = p.basis;
    M.V = S.V;
    M.ldv = (size_t)S.ly.ldv;
    M.L = L;
    M.partials = S.mgs_part;
    M.st = S.dst;
    M.bd_rel = bd_rel;
    M.q = r0;
    M.k = 0;
    M.hcol = S.gv;          // g[0] = beta
    M.vout = S.vec(0);
    M.cur = S.cur;
    M.bar = S.bar + 0;
    CK(launch_mgs(M, s));
    DevState hs;
    if ((rc = S.sync_state(hs))) return rc;
    if (hs.error & 1) return ABG_EDEVICE;
    const double beta = hs.hnext;
    if (!std::isfinite(beta)) return ABG_ENAN;
    if (info) info->beta = beta;
    if (beta == 0.0) {
        if (x0) CK(hipMemcpyAsync(x, x0, (size_t)n * S.sX, hipMemcpyDeviceToDevice, s));
        else CK(launch_combine(p.proj, nullptr, 0.0, p.basis, S.V, S.ly.ldv, 0, S.y, 1.0, x, n,
                               nullptr, nullptr, nullptr, s));
        status = ABG_ZERO_RHS;
        if ((rc = S.literal_residual(b, x))) return rc;
        if ((rc = S.sync_state(hs))) return rc;
        res_final = hs.res;
        goto done;
    }

    {
        double ncp_prev = 0.0, ncp_best = INFINITY;
        int best_k = 0;
        bool finished = false;
        for (int k = 1; k <= k_max && !finished; ++k) {
            // q_k = AB w_k or BA w_k
            if (method == ABG_METHOD_BA) {
                void *z = S.Z ? S.zcol(k - 1) : S.tm;
                if ((rc = S.fwd(S.cur, z))) return rc;
                if ((rc = S.back(z, S.q))) return rc;
            } else {
                if ((rc = S.back(S.cur, S.tn))) return rc;
                if ((rc = S.fwd(S.tn, S.q))) return rc;
            }
            M.q = S.q;
            M.k = k;
            M.hcol = S.H + (size_t)(k - 1) * ld;
            M.vout = S.vec(k);
            M.bar = S.bar + k;
            CK(launch_mgs(M, s));
            if (st.kind == ABG_STOP_NCP && k > 1)
                CK(hipMemcpyAsync(S.yprev, S.y, (size_t)(k - 1) * 8, hipMemcpyDeviceToDevice, s));
            CK(launch_givens(S.H, ld, S.R, S.cs, S.sn, S.gv, S.y,
                             (method == ABG_METHOD_AB && need_res) ? S.rho : nullptr, beta, k, 1,
                             S.dst, s));
            if (need_res) {
                int nb = 0;
                if (method == ABG_METHOD_BA)
                    CK(launch_combine(p.proj, S.rb0, 1.0, p.proj, S.Z, S.ly.mp, k, S.y, -1.0, S.tm,
                                      m, S.part, &nb, S.dst, s));
                else
                    CK(launch_combine(p.proj, nullptr, 0.0, p.basis, S.V, S.ly.ldv, k + 1, S.rho,
                                      1.0, S.tm, m, S.part, &nb, S.dst, s));
                CK(launch_reduce_sqrt(S.part, nb, &S.dst->res, s));
                if (st.kind == ABG_STOP_NCP) CK(launch_ncp(g, p.proj, S.tm, S.ncp, &S.dst->ncp, s));
            }
            if ((rc = S.sync_state(hs))) return rc;
            if (hs.error & 1) return ABG_EDEVICE;
            if ((hs.error & 2) || !std::isfinite(hs.ls)) return ABG_ENAN;
            if (hs.error & 4) return ABG_ENAN;
            k_done = k;
            hist(info ? info->ls_hist : nullptr, k, hs.ls);
            const bool breakdown = hs.breakdown != 0;
            if (st.kind == ABG_STOP_DP) {
                double rk = hs.res;
                if (!std::isfinite(rk)) return ABG_ENAN;
                if (rk <= thr * (1.0 + dp_slack(p.basis))) {
                    // confirm with the explicit residual of x_k
                    if ((rc = S.build_x(S.y, k, x0, x))) return rc;
                    if ((rc = S.literal_residual(b, x))) return rc;
                    DevState h2;
                    if ((rc = S.sync_state(h2))) return rc;
                    ++n_literal;
                    rk = h2.res;
                    if (rk <= thr) {
                        hist(info ? info->res_hist : nullptr, k, rk);
                        k_stop = k;
                        status = ABG_OK;
                        res_final = rk;
                        finished = true;
                        break;
                    }
                }
                hist(info ? info->res_hist : nullptr, k, rk);
            } else if (st.kind == ABG_STOP_NCP) {
                hist(info ? info->res_hist : nullptr, k, hs.res);
                hist(info ? info->ncp_hist : nullptr, k, hs.ncp);
                if (k >= 2 && hs.ncp > ncp_prev) {
                    if ((rc = S.build_x(S.yprev, k - 1, x0, x))) return rc;
                    k_stop = k - 1;
                    ncp_final = ncp_prev;
                    status = ABG_OK;
                    finished = true;
                    break;
                }
                if (hs.ncp < ncp_best) {
                    ncp_best = hs.ncp;
                    best_k = k;
                    CK(hipMemcpyAsync(S.ybest, S.y, (size_t)k * 8, hipMemcpyDeviceToDevice, s));
                }
                ncp_prev = hs.ncp;
            }
            if (breakdown) {
                if ((rc = S.build_x(S.y, k, x0, x))) return rc;
                k_stop = k;
                status = ABG_BREAKDOWN;
                finished = true;
                break;
            }
            if (k == k_max) {
                if (st.kind == ABG_STOP_NCP) {
                    if ((rc = S.build_x(S.ybest, best_k, x0, x))) return rc;
                    k_stop = best_k;
                    ncp_final = ncp_best;
                } else {
                    if ((rc = S.build_x(S.y, k, x0, x))) return rc;
                    k_stop = k;
                    status = st.kind == ABG_STOP_DP ? ABG_NOT_CONVERGED : ABG_OK;
                }
                finished = true;
            }
        }
        // explicit residual of the returned iterate; a NaN/Inf anywhere in b shows here
        if ((rc = S.literal_residual(b, x))) return rc;
        if ((rc = S.sync_state(hs))) return rc;
        res_final = hs.res;
        if (!std::isfinite(res_final)) return ABG_ENAN;
    }

done:
    if (info) {
        info->k_stop = k_stop;
        info->k_done = k_done;
        info->status = status;
        info->n_literal = n_literal;
        info->res_norm = res_final;
        info->ncp_dist = ncp_final;
        if (info->H && k_done > 0) {
            CK(hipMemcpyAsync(info->H, S.H, (size_t)ld * k_max * 8, hipMemcpyDeviceToHost, s));
            CK(hipStreamSynchronize(s));
        }
    }
    if (profiling_on()) profile_flush();
    return status;
}

}  // namespace abg
