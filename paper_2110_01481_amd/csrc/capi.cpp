// extern "C" entry points of libabgmres: argument checking, geometry set-up (angle
// table, Table 6.1 parameters), dispatch to the HIP launchers, and launch timing.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <new>
#include <vector>

#include "abg_internal.h"

namespace abg {
namespace {

std::mutex g_prof_mu;
bool g_prof_on = false;
long long g_prof_count[kProfKinds] = {};
double g_prof_ms[kProfKinds] = {};
struct Pending {
    int kind;
    hipEvent_t e0, e1;
    long long solve;   // solve id of the launching thread (0: outside a solve)
    int step;
};
std::atomic<long long> g_solve_ids{0};
thread_local long long t_solve = 0;
thread_local bool t_prof_suppressed = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_event_pool;   // recycled so timing adds no event creation

hipEvent_t take_event()
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

bool valid_dtype_proj(int t) { return t == ABG_F64 || t == ABG_F32; }

int current_device_matches(const Geometry &g)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return ABG_EHIP;
    return dev == g.device ? ABG_OK : ABG_EINVAL;
}

AngleParams make_angle(double theta_deg, double ds)
{
    AngleParams P{};
    const double rad = theta_deg * (M_PI / 180.0);
    double c = std::cos(rad), s = std::sin(rad);
    if (std::fmod(theta_deg, 90.0) == 0.0) {
        long long quadrant = std::llround(theta_deg / 90.0);
        quadrant = ((quadrant % 4) + 4) % 4;
        static const double cq[4] = {1.0, 0.0, -1.0, 0.0};
        static const double sq[4] = {0.0, 1.0, 0.0, -1.0};
        c = cq[quadrant];
        s = sq[quadrant];
    }
    P.c = c;
    P.s = s;
    P.p = std::fmax(std::fabs(c), std::fabs(s));
    P.q = std::fmin(std::fabs(c), std::fabs(s));
    P.steep = std::fabs(c) >= std::fabs(s) ? 1 : 0;
    P.m = P.steep ? -s / c : -c / s;
    P.inv = P.steep ? 1.0 / c : 1.0 / s;
    P.len = 1.0 / P.p;
    P.axis = P.q == 0.0 ? 1 : 0;
    P.invq = P.axis ? 0.0 : 1.0 / P.q;
    if (P.axis) P.m = 0.0;
    P.cu = c / ds;
    P.su = s / ds;
    P.half = 0.5 * (P.p + P.q);
    P.invpq = P.axis ? 0.0 : 1.0 / (P.p * P.q);
    return P;
}

}  // namespace

bool profiling_on() { return g_prof_on; }

ProfScope::ProfScope(int kind_, hipStream_t s_, int step_, bool ext_)
    : kind(kind_), step(step_), s(s_), ext(ext_)
{
    if (!g_prof_on || t_prof_suppressed) return;
    e0 = take_event();
    e1 = take_event();
    if (!e0 || !e1) {
        e0 = e1 = nullptr;
        return;
    }
    if (!ext) (void)hipEventRecord(e0, s);
}

namespace {
// Launches whose events are read only when the counters are (or when this many wait):
// reading them at the end of every solve would stall the host between solves.
constexpr size_t kMaxPending = 4096;
void flush_locked();
}  // namespace

ProfScope::~ProfScope()
{
    if (!e0) return;
    if (!ext) (void)hipEventRecord(e1, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_pending.push_back({kind, e0, e1, t_solve, step});
    if (g_pending.size() >= kMaxPending) flush_locked();
}

ProfSuppress::ProfSuppress() : prev(t_prof_suppressed) { t_prof_suppressed = true; }
ProfSuppress::~ProfSuppress() { t_prof_suppressed = prev; }

void profile_solve_begin()
{
    if (!g_prof_on) return;
    t_solve = ++g_solve_ids;
}

namespace {
// Removes pending launches of the current solve selected by `pred` (caller holds the lock).
template <typename Pred>
void drop_pending(long long id, Pred pred)
{
    std::vector<Pending> keep;
    keep.reserve(g_pending.size());
    for (auto &p : g_pending) {
        if (p.solve == id && p.step > 0 && pred(p.step)) {
            (void)hipEventSynchronize(p.e1);
            g_event_pool.push_back(p.e0);
            g_event_pool.push_back(p.e1);
        } else {
            keep.push_back(p);
        }
    }
    g_pending.swap(keep);
}
}  // namespace

void profile_solve_end(int last_step)
{
    const long long id = t_solve;
    t_solve = 0;
    if (!g_prof_on || id == 0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    drop_pending(id, [&](int step) { return step > last_step; });
}

void profile_drop_step(int step)
{
    if (!g_prof_on || t_solve == 0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    drop_pending(t_solve, [&](int st) { return st == step; });
}

namespace {
// Accumulates the durations of all pending launches (caller holds the lock).
void flush_locked()
{
    for (auto &p : g_pending) {
        float ms = 0.f;
        (void)hipEventSynchronize(p.e1);
        if (hipEventElapsedTime(&ms, p.e0, p.e1) == hipSuccess) {
            g_prof_ms[p.kind] += ms;
            g_prof_count[p.kind] += 1;
        }
        g_event_pool.push_back(p.e0);
        g_event_pool.push_back(p.e1);
    }
    g_pending.clear();
}
}  // namespace

void profile_flush()
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    flush_locked();
}

}  // namespace abg

using namespace abg;

extern "C" {

int abg_create_geometry(int N, int n_ang, double ang_start_deg, double ang_range_deg,
                        const double *angles_deg, int n_det, double det_spacing,
                        abg_geometry **out)
{
    if (!out) return ABG_EINVAL;
    *out = nullptr;
    if (N < 1 || N > 32768 || n_ang < 1 || n_det < 1 || n_det > (1 << 24)) return ABG_EINVAL;
    if (!(det_spacing >= 0.75 && det_spacing <= 64.0)) return ABG_EINVAL;
    if (!angles_deg && !(std::isfinite(ang_start_deg) && std::isfinite(ang_range_deg)))
        return ABG_EINVAL;
    abg_geometry *h = new (std::nothrow) abg_geometry;
    if (!h) return ABG_ENOMEM;
    Geometry &g = h->g;
    g.N = N;
    g.n_ang = n_ang;
    g.n_det = n_det;
    g.ds = det_spacing;
    g.theta.resize(n_ang);
    g.host.resize(n_ang);
    for (int a = 0; a < n_ang; ++a) {
        const double th = angles_deg ? angles_deg[a]
                                     : ang_start_deg + ((double)a * ang_range_deg) / n_ang;
        if (!std::isfinite(th)) {
            delete h;
            return ABG_EINVAL;
        }
        g.theta[a] = th;
        g.host[a] = make_angle(th, det_spacing);
    }
    if (hipGetDevice(&g.device) != hipSuccess ||
        hipMalloc((void **)&g.dev, sizeof(AngleParams) * n_ang) != hipSuccess) {
        delete h;
        return ABG_EHIP;
    }
    if (hipMemcpy(g.dev, g.host.data(), sizeof(AngleParams) * n_ang, hipMemcpyHostToDevice) !=
        hipSuccess) {
        (void)hipFree(g.dev);
        delete h;
        return ABG_EHIP;
    }
    *out = h;
    return ABG_OK;
}

int abg_destroy_geometry(abg_geometry *h)
{
    if (!h) return ABG_OK;
    int rc = ABG_OK;
    if (h->g.dev && hipFree(h->g.dev) != hipSuccess) rc = ABG_EHIP;
    ncp_release(h->g);
    delete h;
    return rc;
}

namespace {

// Strip-model weight (area of pixel and strip over ds) of a pixel whose centre lies e >= 0
// from the ray (detector units), for an angle with p = max(|cos|,|sin|), q = min(...):
// the integral of the line-model trapezoid over the strip.
double trapezoid_below(double a, const AngleParams &P)
{
    const double h0 = P.p - P.half, h1 = P.half;
    if (a >= h1) return 0.0;
    if (a >= h0) return (h1 - a) * (h1 - a) * 0.5 * P.invpq;
    return 0.5 * P.q * P.len + (h0 - a) * P.len;
}

double strip_weight(double e, const AngleParams &P, double ds)
{
    const double lo = e - 0.5 * ds, hi = e + 0.5 * ds;
    const double glo = lo >= 0.0 ? trapezoid_below(lo, P) : 1.0 - trapezoid_below(-lo, P);
    return (glo - trapezoid_below(hi, P)) / ds;
}

// Largest strip-model entry. An angle's entries are at most its weight at e = 0 (the weight
// falls with e), so angles are visited in decreasing order of that bound and the scan
// stops once no remaining angle can exceed the maximum found; each visited angle takes
// every pixel at its nearest bin.
double strip_max_entry(const Geometry &g)
{
    std::vector<std::pair<double, int>> order(g.n_ang);
    for (int a = 0; a < g.n_ang; ++a) order[a] = {strip_weight(0.0, g.host[a], g.ds), a};
    std::sort(order.begin(), order.end(), [](const auto &u, const auto &v) { return u.first > v.first; });
    const double s0 = -0.5 * (g.n_det - 1) * g.ds;
    double best = 0.0;
    for (const auto &oa : order) {
        if (oa.first <= best) break;
        const AngleParams &P = g.host[oa.second];
        for (int r = 0; r < g.N; ++r) {
            const double yc = r - 0.5 * g.N + 0.5;
            for (int c = 0; c < g.N; ++c) {
                const double t0 = (c - 0.5 * g.N + 0.5) * P.c + yc * P.s;
                long long i = std::llround((t0 - s0) / g.ds);
                i = std::min<long long>(std::max<long long>(i, 0), g.n_det - 1);
                best = std::max(best, strip_weight(std::fabs(s0 + i * g.ds - t0), P, g.ds));
            }
        }
    }
    return best;
}

}  // namespace

int abg_geometry_set_strip_threshold(abg_geometry *h, double tau, double *max_entry)
{
    if (!h || !(tau >= 0.0 && tau <= 1.0) || !(h->g.ds <= 1.4)) return ABG_EINVAL;
    if (h->g.strip_max <= 0.0) h->g.strip_max = strip_max_entry(h->g);
    h->g.tau_thr = (tau - 1e-6) * h->g.strip_max;
    if (max_entry) *max_entry = h->g.strip_max;
    return ABG_OK;
}

int abg_geometry_set_model(abg_geometry *h, int fp_model)
{
    if (!h || fp_model < ABG_FP_LINE || fp_model > ABG_FP_JOSEPH) return ABG_EINVAL;
    if (fp_model == ABG_FP_STRIP && !(h->g.ds <= 1.4)) return ABG_EINVAL;
    h->g.model = fp_model;
    return ABG_OK;
}

int abg_geometry_get_model(const abg_geometry *h, int *fp_model)
{
    if (!h || !fp_model) return ABG_EINVAL;
    *fp_model = h->g.model;
    return ABG_OK;
}

int abg_geometry_sizes(const abg_geometry *h, long long *n, long long *m)
{
    if (!h) return ABG_EINVAL;
    if (n) *n = h->g.n();
    if (m) *m = h->g.m();
    return ABG_OK;
}

size_t abg_fp_workspace_bytes(const abg_geometry *h, int dtype)
{
    if (!h || !valid_dtype_proj(dtype)) return 0;
    return fp_workspace_bytes(h->g, dtype);
}

int abg_fp_apply(const abg_geometry *h, int dtype, const void *x, void *y, void *ws,
                 size_t ws_bytes, void *stream)
{
    if (!h || !x || !y || !ws || !valid_dtype_proj(dtype)) return ABG_EINVAL;
    if (reinterpret_cast<uintptr_t>(ws) % 256) return ABG_EINVAL;
    if (ws_bytes < fp_workspace_bytes(h->g, dtype)) return ABG_ENOMEM;
    int rc = current_device_matches(h->g);
    if (rc) return rc;
    return launch_forward(h->g, dtype, x, y, ws, static_cast<hipStream_t>(stream)) == hipSuccess
               ? ABG_OK
               : ABG_EHIP;
}

int abg_fp_apply_noalloc(const abg_geometry *h, int dtype, const void *x, void *y, void *stream)
{
    if (!h || !x || !y || !valid_dtype_proj(dtype)) return ABG_EINVAL;
    int rc = current_device_matches(h->g);
    if (rc) return rc;
    return fp_apply_static(h->g, dtype, x, y, static_cast<hipStream_t>(stream));
}

int abg_bp_apply(const abg_geometry *h, int kind, int dtype, const void *y, void *x,
                 void *stream)
{
    if (!h || !x || !y || !valid_dtype_proj(dtype)) return ABG_EINVAL;
    if (kind < ABG_BP_HAT || kind > ABG_BP_STRIP_TAU) return ABG_EINVAL;
    if (kind == ABG_BP_STRIP_TAU && !(h->g.ds <= 1.4)) return ABG_EINVAL;
    int rc = current_device_matches(h->g);
    if (rc) return rc;
    return launch_back(h->g, kind, dtype, y, x, static_cast<hipStream_t>(stream)) == hipSuccess
               ? ABG_OK
               : ABG_EHIP;
}

static int check_solver_args(const abg_geometry *h, int method, int k_max, abg_precision p,
                             abg_stop st)
{
    if (!h) return ABG_EINVAL;
    if (method != ABG_METHOD_AB && method != ABG_METHOD_BA) return ABG_EINVAL;
    if (k_max < 1 || k_max > 500) return ABG_EINVAL;
    if (!valid_dtype_proj(p.proj)) return ABG_EINVAL;
    if (p.basis != ABG_F64 && p.basis != ABG_F32 && p.basis != ABG_BF16) return ABG_EINVAL;
    if (dtype_size(p.basis) > dtype_size(p.proj)) return ABG_EINVAL;
    if (st.kind == ABG_STOP_DP) {
        if (!(st.tau >= 1.0) || !(st.noise_norm > 0.0) || !std::isfinite(st.tau * st.noise_norm))
            return ABG_EINVAL;
    } else if (st.kind == ABG_STOP_NCP) {
        if (h->g.n_det < 2 || h->g.n_det / 2 > 2048) return ABG_EINVAL;
    } else if (st.kind != ABG_STOP_NONE) {
        return ABG_EINVAL;
    }
    return ABG_OK;
}

size_t abg_workspace_bytes(const abg_geometry *h, int method, int k_max, abg_precision p,
                           abg_stop st)
{
    if (check_solver_args(h, method, k_max, p, st) != ABG_OK) return 0;
    return solver_workspace_bytes(h->g, method, k_max, p, st);
}

static int solve_entry(int method, const abg_geometry *h, int bp_kind, const void *b,
                       const void *x0, void *x, int k_max, abg_stop st, abg_precision p,
                       void *ws, size_t ws_bytes, abg_info *info, void *stream)
{
    int rc = check_solver_args(h, method, k_max, p, st);
    if (rc) return rc;
    if (bp_kind < ABG_BP_HAT || bp_kind > ABG_BP_STRIP_TAU) return ABG_EINVAL;
    if (bp_kind == ABG_BP_STRIP_TAU && !(h->g.ds <= 1.4)) return ABG_EINVAL;
    if (!b || !x || !ws || x == b || (x0 && x == x0)) return ABG_EINVAL;
    if (reinterpret_cast<uintptr_t>(ws) % 256) return ABG_EINVAL;
    if ((rc = current_device_matches(h->g))) return rc;
    rc = run_solver(h->g, method, bp_kind, b, x0, x, k_max, st, p, ws, ws_bytes, info,
                    static_cast<hipStream_t>(stream));
    if (info) info->status = rc;
    return rc;
}

int abg_ab_gmres(const abg_geometry *h, int bp_kind, const void *b, const void *x0, void *x,
                 int k_max, abg_stop st, abg_precision p, void *ws, size_t ws_bytes,
                 abg_info *info, void *stream)
{
    return solve_entry(ABG_METHOD_AB, h, bp_kind, b, x0, x, k_max, st, p, ws, ws_bytes, info,
                       stream);
}

int abg_ba_gmres(const abg_geometry *h, int bp_kind, const void *b, const void *x0, void *x,
                 int k_max, abg_stop st, abg_precision p, void *ws, size_t ws_bytes,
                 abg_info *info, void *stream)
{
    return solve_entry(ABG_METHOD_BA, h, bp_kind, b, x0, x, k_max, st, p, ws, ws_bytes, info,
                       stream);
}

int abg_gmres_error_history(const abg_geometry *h, int method, int bp_kind, int k_max,
                            abg_stop st, abg_precision p, const void *x0, const void *x_ref,
                            void *ws, size_t ws_bytes, int k_done, double *err, void *stream)
{
    int rc = check_solver_args(h, method, k_max, p, st);
    if (rc) return rc;
    if (bp_kind < ABG_BP_HAT || bp_kind > ABG_BP_STRIP_TAU) return ABG_EINVAL;
    if (!x_ref || !ws || (k_done > 0 && !err)) return ABG_EINVAL;
    if (reinterpret_cast<uintptr_t>(ws) % 256) return ABG_EINVAL;
    if ((rc = current_device_matches(h->g))) return rc;
    return gmres_error_history(h->g, method, bp_kind, k_max, st, p, ws, ws_bytes, x0, x_ref,
                               k_done, err, static_cast<hipStream_t>(stream));
}

// ---- batched engine ------------------------------------------------------------------

size_t abg_request_bytes(const abg_geometry *h, int method, int k_max, abg_precision p,
                         abg_stop st)
{
    return abg_workspace_bytes(h, method, k_max, p, st);
}

int abg_engine_create(abg_precision p, int max_slots, void *stream, abg_engine **out)
{
    if (!out) return ABG_EINVAL;
    *out = nullptr;
    abg_engine *h = new (std::nothrow) abg_engine{nullptr};
    if (!h) return ABG_EHIP;
    const int rc = engine_create(p, max_slots, static_cast<hipStream_t>(stream), &h->e);
    if (rc != ABG_OK) {
        delete h;
        return rc;
    }
    *out = h;
    return ABG_OK;
}

int abg_engine_destroy(abg_engine *h)
{
    if (!h) return ABG_OK;
    engine_destroy(h->e);
    delete h;
    return ABG_OK;
}

int abg_engine_submit(abg_engine *h, const abg_request *r)
{
    if (!h || !r) return ABG_EINVAL;
    if (r->stop.kind == ABG_STOP_NCP) return ABG_EINVAL;
    abg_precision p;
    engine_precision(h->e, &p);
    int rc = check_solver_args(r->g, r->method, r->k_max, p, r->stop);
    if (rc) return rc;
    if (r->bp_kind != ABG_BP_HAT && r->bp_kind != ABG_BP_ADJ) return ABG_EINVAL;
    if (r->g->g.model != ABG_FP_LINE) return ABG_EINVAL;
    if (!r->b || !r->x || !r->ws || r->x == r->b || (r->x0 && r->x == r->x0)) return ABG_EINVAL;
    if (reinterpret_cast<uintptr_t>(r->ws) % 256) return ABG_EINVAL;
    if (r->g->g.device != engine_device(h->e)) return ABG_EINVAL;
    if ((rc = current_device_matches(r->g->g))) return rc;
    if (r->ws_bytes < solver_workspace_bytes(r->g->g, r->method, r->k_max, p, r->stop))
        return ABG_ENOMEM;
    return engine_submit(h->e, r->g->g, *r);
}

int abg_engine_step(abg_engine *h, int *n_active)
{
    if (!h) return ABG_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return ABG_EHIP;
    if (dev != engine_device(h->e)) return ABG_EINVAL;
    return engine_step(h->e, n_active);
}

int abg_engine_poll(abg_engine *h, long long *tags, int *status, int max, int *n)
{
    if (!h || !n || max < 0) return ABG_EINVAL;
    return engine_poll(h->e, tags, status, max, n);
}

int abg_engine_set_tiles(abg_engine *h, int rays, int ang_block, int sched)
{
    if (!h) return ABG_EINVAL;
    return engine_set_tiles(h->e, rays, ang_block, sched);
}

int abg_engine_get_tiles(const abg_engine *h, int *rays, int *ang_block, int *sched)
{
    if (!h || !rays || !ang_block || !sched) return ABG_EINVAL;
    return engine_get_tiles(h->e, rays, ang_block, sched);
}

int abg_engine_autotune(abg_engine *h, int reps, int *rays, int *ang_block, int *sched,
                        double *ms)
{
    if (!h || !rays || !ang_block || !sched || !ms || reps < 1 || reps > 1000) return ABG_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return ABG_EHIP;
    if (dev != engine_device(h->e)) return ABG_EINVAL;
    return engine_autotune(h->e, reps, rays, ang_block, sched, ms);
}

int abg_batch_solve(const abg_request *r, int n, abg_precision p, int rays, int ang_block,
                    int sched, void *stream)
{
    if (n < 0 || (n > 0 && !r)) return ABG_EINVAL;
    if (n == 0) return ABG_OK;
    abg_engine *h = nullptr;
    int rc = abg_engine_create(p, n, stream, &h);
    if (rc) return rc;
    int cur_rays = 0, cur_ab = 0, cur_sched = 0;
    abg_engine_get_tiles(h, &cur_rays, &cur_ab, &cur_sched);
    if ((rays > 0 || ang_block > 0 || sched >= 0) &&
        (rc = abg_engine_set_tiles(h, rays > 0 ? rays : cur_rays,
                                   ang_block > 0 ? ang_block : cur_ab,
                                   sched >= 0 ? sched : cur_sched))) {
        abg_engine_destroy(h);
        return rc;
    }
    for (int i = 0; i < n && rc == ABG_OK; ++i) rc = abg_engine_submit(h, &r[i]);
    int first_err = rc;
    int active = n;
    std::vector<long long> tags(n);
    std::vector<int> st(n);
    // every round advances a running problem or settles a pending decision: bound the
    // loop well above what the iteration caps allow
    long long guard = 16;
    for (int i = 0; i < n; ++i) guard += 4LL * (r[i].k_max + 4);
    while (first_err == ABG_OK && active > 0) {
        rc = abg_engine_step(h, &active);
        if (rc) first_err = rc;
        if (--guard < 0) first_err = ABG_EDEVICE;
    }
    int got = 0;
    if (first_err == ABG_OK) {
        rc = abg_engine_poll(h, tags.data(), st.data(), n, &got);
        if (rc) first_err = rc;
        for (int i = 0; i < got && first_err == ABG_OK; ++i)
            if (st[i] < 0) first_err = st[i];
    }
    abg_engine_destroy(h);
    return first_err;
}

int abg_mgs_force_stream(int on)
{
    set_mgs_force_stream(on);
    return ABG_OK;
}

size_t abg_lsq_workspace_bytes(const abg_geometry *h, int method, int dtype)
{
    if (!h || (method != ABG_METHOD_LSQR && method != ABG_METHOD_LSMR) || !valid_dtype_proj(dtype))
        return 0;
    return lsq_workspace_bytes(h->g, method, dtype);
}

static int lsq_entry(int method, const abg_geometry *h, const void *b, const void *x0, void *x,
                     int k_max, abg_stop st, int dtype, void *ws, size_t ws_bytes, abg_info *info,
                     const void *x_ref, double *err_hist, void *stream)
{
    if (!h || !valid_dtype_proj(dtype) || k_max < 1 || k_max > 500) return ABG_EINVAL;
    if (st.kind == ABG_STOP_DP) {
        if (!(st.tau >= 1.0) || !(st.noise_norm > 0.0) || !std::isfinite(st.tau * st.noise_norm))
            return ABG_EINVAL;
    } else if (st.kind == ABG_STOP_NCP) {
        if (h->g.n_det < 2 || h->g.n_det / 2 > 2048) return ABG_EINVAL;
    } else if (st.kind != ABG_STOP_NONE) {
        return ABG_EINVAL;
    }
    if (!b || !x || !ws || x == b || (x0 && x == x0)) return ABG_EINVAL;
    if ((x_ref == nullptr) != (err_hist == nullptr) || (x_ref && x_ref == x)) return ABG_EINVAL;
    if (reinterpret_cast<uintptr_t>(ws) % 256) return ABG_EINVAL;
    int rc = current_device_matches(h->g);
    if (rc) return rc;
    rc = run_lsq(h->g, method, b, x0, x, k_max, st, dtype, ws, ws_bytes, info, x_ref, err_hist,
                 static_cast<hipStream_t>(stream));
    if (info) info->status = rc;
    return rc;
}

int abg_lsqr(const abg_geometry *h, const void *b, const void *x0, void *x, int k_max, abg_stop st,
             int dtype, void *ws, size_t ws_bytes, abg_info *info, const void *x_ref,
             double *err_hist, void *stream)
{
    return lsq_entry(ABG_METHOD_LSQR, h, b, x0, x, k_max, st, dtype, ws, ws_bytes, info, x_ref,
                     err_hist, stream);
}

int abg_lsmr(const abg_geometry *h, const void *b, const void *x0, void *x, int k_max, abg_stop st,
             int dtype, void *ws, size_t ws_bytes, abg_info *info, const void *x_ref,
             double *err_hist, void *stream)
{
    return lsq_entry(ABG_METHOD_LSMR, h, b, x0, x, k_max, st, dtype, ws, ws_bytes, info, x_ref,
                     err_hist, stream);
}

const char *abg_status_string(int status)
{
    switch (status) {
    case ABG_OK: return "ok";
    case ABG_EINVAL: return "invalid argument";
    case ABG_ENOMEM: return "workspace too small";
    case ABG_EHIP: return "HIP runtime error";
    case ABG_ENAN: return "NaN or Inf in a norm";
    case ABG_EDEVICE: return "device-side wait exceeded its bound";
    case ABG_EFULL: return "no free slot in the engine";
    case ABG_NOT_CONVERGED: return "discrepancy principle not met by k_max";
    case ABG_BREAKDOWN: return "Arnoldi breakdown (Krylov space exhausted)";
    case ABG_ZERO_RHS: return "zero initial residual";
    default: return "unknown status";
    }
}

int abg_profile_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    // events for every launch that can be pending, created now rather than in the solves
    while (g_prof_on && g_event_pool.size() < 2 * kMaxPending + 64) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return ABG_EHIP;
        g_event_pool.push_back(e);
    }
    return ABG_OK;
}

int abg_ncp_force_goertzel(int on)
{
    ncp_force_goertzel(on);
    return ABG_OK;
}

int abg_fp_force_block_shape(int lg_angles)
{
    if (lg_angles < -1 || lg_angles > 2) return ABG_EINVAL;
    fwd_force_block_shape(lg_angles);
    return ABG_OK;
}

int abg_fp_force_stage_share(int eighths)
{
    if (eighths < -1 || eighths > 8) return ABG_EINVAL;
    fwd_force_stage_eighths(eighths);
    return ABG_OK;
}

int abg_release_process_resources(void)
{
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        flush_locked();
        g_prof_on = false;
        for (hipEvent_t e : g_event_pool) (void)hipEventDestroy(e);
        g_event_pool.clear();
        g_event_pool.shrink_to_fit();
    }
    return host_release_all();
}

int abg_profile_read(long long counts[ABG_PROF_KINDS], double ms[ABG_PROF_KINDS], int reset)
{
    static_assert(ABG_PROF_KINDS == kProfKinds, "profile kinds");
    profile_flush();
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (int i = 0; i < kProfKinds; ++i) {
        if (counts) counts[i] = g_prof_count[i];
        if (ms) ms[i] = g_prof_ms[i];
        if (reset) {
            g_prof_count[i] = 0;
            g_prof_ms[i] = 0.0;
        }
    }
    return ABG_OK;
}

}  // extern "C"
