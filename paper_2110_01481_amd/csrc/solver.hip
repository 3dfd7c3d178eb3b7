// AB-GMRES and BA-GMRES drivers (Sec. 2) with discrepancy-principle and NCP stopping
// (Sec. 6.3). The host thread sequences kernels; every vector operation runs in the
// kernels of this library.
//
// Step k (BA):  z = A w_k (column k of Z when a stopping rule needs the residual),
//               q = B z, MGS, Givens, then r_k = (b - A x_0) - Z y_k.
// Step k (AB):  t = B w_k, q = A t, MGS, Givens, then r_k = W_{k+1}(||r_0|| e_1 - H_k y_k).
// Both residual forms equal b - A x_k by linearity and the Arnoldi relation; the
// discrepancy principle confirms a candidate stop with the explicit b - A x_k.
//
// Pipelining: the host enqueues step k+1 before it waits for step k's scalars. Stops are
// decided on the device by the last kernel of a step (DP candidate, NCP increase) or by
// MGS (breakdown); the kernels of every later step then return at entry, so a step that
// was enqueued past the stop costs only its launches. y_k is kept for every k, so the
// iterate of any step can be formed afterwards.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "abg_internal.h"

namespace abg {
namespace {

struct Layout {
    size_t V, Z, cur, q, rb0, tm, tn, fpws, H, R, cs, sn, g, Y, rho;
    size_t part, mgs_part, tick, count, st, ncp, q64, gram, total;
    long long L, ldv, mp, np;
    int mgs_rows;
    long long mgs_cap;
};

long long round_up(long long v, long long a) { return (v + a - 1) / a * a; }

Layout make_layout(const Geometry &g, int method, int k_max, abg_precision p, abg_stop st)
{
    Layout ly{};
    const size_t sX = dtype_size(p.proj), sV = dtype_size(p.basis);
    ly.mp = round_up(g.m(), kVecPad);
    ly.np = round_up(g.n(), kVecPad);
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
    ly.Y = take((size_t)k_max * k_max * 8);
    ly.rho = take((ld + 1) * 8);
    ly.part = take(2048 * 8);
    // MGS slot tables: two of (2 k_max + 3) rows (the low-synchronisation form uses rows
    // 0..2k), one column per block of the largest group
    ly.mgs_rows = 2 * k_max + 3;
    const long long gmax = std::min<long long>(kMaxGrid, (ly.L + 255) / 256);
    ly.mgs_cap = 2LL * ly.mgs_rows * gmax;
    ly.mgs_part = take((size_t)ly.mgs_cap * 8);
    ly.tick = take((ld + 2) * 4);
    ly.q64 = ly.L > kRegMaxL ? take((size_t)ly.ldv * 8) : 0;
    ly.gram = take(gram_entries(k_max) * 8);
    ly.count = take(64);
    ly.st = take(sizeof(DevState));
    ly.ncp = st.kind == ABG_STOP_NCP ? take(ncp_scratch_bytes(g)) : 0;
    ly.total = off;
    return ly;
}

constexpr int kRing = 4;

// Pinned scalar slots and step events of a solve. They are pooled process-wide
// (allocating pinned memory and events on every call costs more than a short solve): a
// solve leases one set for its duration and returns it when it ends; host_release_all
// frees the idle sets (abg_release_process_resources).
struct HostRes {
    DevState *slots = nullptr;
    DevState *dslots = nullptr;   // the same slots as the device addresses them
    int capacity = 0;
    int device = -1;
    hipEvent_t ev[kRing] = {};
};

std::mutex g_host_mu;
std::vector<HostRes> g_host_idle;

void host_free(HostRes &h)
{
    if (h.slots) (void)hipHostFree(h.slots);
    for (auto &ev : h.ev)
        if (ev) (void)hipEventDestroy(ev);
    h = HostRes{};
}

}  // namespace

int host_release_all()
{
    std::lock_guard<std::mutex> lk(g_host_mu);
    int prev = -1;
    (void)hipGetDevice(&prev);
    for (auto &h : g_host_idle) {
        // events and pinned memory are released with their device current
        if (h.device >= 0) (void)hipSetDevice(h.device);
        host_free(h);
    }
    g_host_idle.clear();
    if (prev >= 0) (void)hipSetDevice(prev);
    return ABG_OK;
}

namespace {

struct HostLease {
    HostRes r;
    hipStream_t s = nullptr;
    bool held = false;

    // an idle set of the current device (the smallest that holds k_max + 1 slots, else
    // any, grown), or a new one
    hipError_t acquire(int k_max, hipStream_t s_)
    {
        s = s_;
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        {
            std::lock_guard<std::mutex> lk(g_host_mu);
            int pick = -1;
            for (int i = 0; i < (int)g_host_idle.size(); ++i) {
                const HostRes &h = g_host_idle[i];
                if (h.device != dev) continue;
                if (pick < 0) pick = i;
                const int cp = g_host_idle[pick].capacity;
                const bool fits = h.capacity >= k_max + 1, pfits = cp >= k_max + 1;
                if ((fits && (!pfits || h.capacity < cp)) || (!fits && !pfits && h.capacity > cp))
                    pick = i;
            }
            if (pick >= 0) {
                r = g_host_idle[pick];
                g_host_idle.erase(g_host_idle.begin() + pick);
            }
        }
        held = true;
        if (r.device != dev) {
            r.device = dev;
            for (auto &ev : r.ev) {
                e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
                if (e != hipSuccess) return e;
            }
        }
        if (r.capacity < k_max + 1) {
            if (r.slots) (void)hipHostFree(r.slots);
            r.slots = r.dslots = nullptr;
            r.capacity = 0;
            e = hipHostMalloc((void **)&r.slots, sizeof(DevState) * (k_max + 1), hipHostMallocDefault);
            if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&r.dslots, r.slots, 0);
            if (e != hipSuccess) return e;
            r.capacity = k_max + 1;
        }
        return hipSuccess;
    }

    // Back to the pool once the stream is idle (an error return may leave the solve's
    // kernels in flight, and they write these slots).
    ~HostLease()
    {
        if (!held) return;
        (void)hipStreamSynchronize(s);
        if (r.slots && r.dslots && r.ev[kRing - 1]) {
            std::lock_guard<std::mutex> lk(g_host_mu);
            g_host_idle.push_back(r);
        } else {
            host_free(r);
        }
    }
};

struct Solve;

// A single solve's share of the device for its Gram-Schmidt block groups (see
// GroupBudget), held from before its first launch until its stream is idle again.
struct GroupHold {
    long long units = 0;
    hipStream_t s = nullptr;
    hipError_t acquire(const Solve &S);
    ~GroupHold()
    {
        if (units <= 0) return;
        (void)hipStreamSynchronize(s);
        device_group_budget().release(units);
    }
};

#define CK(expr)                                   \
    do {                                           \
        hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) return ABG_EHIP;     \
    } while (0)

#define RC(expr)                                   \
    do {                                           \
        int r_ = (expr);                           \
        if (r_ != ABG_OK) return r_;               \
    } while (0)

struct Solve {
    const Geometry &g;
    int method, kind, k_max, ld;
    abg_stop st;
    abg_precision p;
    hipStream_t s;
    Layout ly;
    char *W;
    void *V, *Z, *cur, *q, *rb0, *tm, *tn, *fpws;
    double *H, *R, *cs, *sn, *gv, *Y, *rho, *part, *mgs_part, *q64, *gram;
    unsigned *count, *tick;
    DevState *dst;
    double *ncp;
    HostLease lease;
    HostRes &hr = lease.r;
    size_t sX;
    bool need_res;
    double bd_rel;

    Solve(const Geometry &g_, int method_, int kind_, int k_max_, abg_stop st_,
          abg_precision p_, hipStream_t s_, void *ws)
        : g(g_), method(method_), kind(kind_), k_max(k_max_), ld(k_max_ + 1), st(st_), p(p_),
          s(s_)
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
        Y = reinterpret_cast<double *>(W + ly.Y);
        rho = reinterpret_cast<double *>(W + ly.rho);
        part = reinterpret_cast<double *>(W + ly.part);
        mgs_part = reinterpret_cast<double *>(W + ly.mgs_part);
        count = reinterpret_cast<unsigned *>(W + ly.count);
        tick = reinterpret_cast<unsigned *>(W + ly.tick);
        q64 = ly.q64 ? reinterpret_cast<double *>(W + ly.q64) : nullptr;
        gram = reinterpret_cast<double *>(W + ly.gram);
        dst = reinterpret_cast<DevState *>(W + ly.st);
        ncp = ly.ncp ? reinterpret_cast<double *>(W + ly.ncp) : nullptr;
        sX = dtype_size(p.proj);
        need_res = st.kind != ABG_STOP_NONE;
        bd_rel = (p.basis == ABG_F64 && p.proj == ABG_F64) ? 1e-14 : 1e-6;
    }

    char *vec(int i) const { return static_cast<char *>(V) + (size_t)i * ly.ldv * dtype_size(p.basis); }
    char *zcol(int i) const { return static_cast<char *>(Z) + (size_t)i * ly.mp * sX; }
    double *ycol(int k) const { return Y + (size_t)(k - 1) * k_max; }

    // the padding of the forward projector's scratch is zeroed once per solve
    int fwd(const void *x, void *yv, const DevState *sst = nullptr, int k = 0)
    {
        CK(launch_forward(g, p.proj, x, yv, fpws, s, sst, k, true));
        return ABG_OK;
    }
    int back(const void *yv, void *x, const DevState *sst = nullptr, int k = 0)
    {
        CK(launch_back(g, kind, p.proj, yv, x, s, sst, k));
        return ABG_OK;
    }

    MgsLaunch mgs_args(const void *qin, int k) const
    {
        MgsLaunch M{};
        M.tx = p.proj;
        M.tv = p.basis;
        M.V = V;
        M.ldv = (size_t)ly.ldv;
        M.L = ly.L;
        M.partials = mgs_part;
        M.st = dst;
        M.bd_rel = bd_rel;
        M.q = qin;
        M.k = k;
        M.step = k;
        M.hcol = k == 0 ? gv : H + (size_t)(k - 1) * ld;
        M.vout = vec(k);
        M.cur = cur;
        M.rows = ly.mgs_rows;
        M.ticket = tick + k;
        M.q64 = q64;
        M.gram = gram;
        return M;
    }

    // Gram-Schmidt of step k followed by its Givens update in the same launch
    MgsLaunch mgs_givens_args(const void *qin, int k, DevState *snap) const
    {
        MgsLaunch M = mgs_args(qin, k);
        M.giv_H = H;
        M.giv_R = R;
        M.giv_cs = cs;
        M.giv_sn = sn;
        M.giv_g = gv;
        M.giv_y = ycol(k);
        M.giv_rho = (method == ABG_METHOD_AB && need_res) ? rho : nullptr;
        M.giv_ld = ld;
        M.snap = snap;
        return M;
    }

    // All kernels of Arnoldi step k, then a copy of the scalars into slot k.
    int enqueue_step(int k)
    {
        if (method == ABG_METHOD_BA) {
            void *z = Z ? zcol(k - 1) : tm;
            RC(fwd(cur, z, dst, k));
            RC(back(z, q, dst, k));
        } else {
            // t = B w_k lands directly in the forward projector's padded copies
            CK(launch_back_staged(g, kind, p.proj, cur, fpws, s, dst, k));
            CK(launch_forward_staged(g, p.proj, q, fpws, s, dst, k));
        }
        // the step's last kernel copies the scalars into host slot k
        DevState *snap = hr.dslots + k;
        const bool ncp_stop = st.kind == ABG_STOP_NCP;
        CK(launch_mgs(mgs_givens_args(q, k, need_res ? nullptr : snap), s));
        if (need_res) {
            DevState *csnap = ncp_stop ? nullptr : snap;
            if (method == ABG_METHOD_BA)
                CK(launch_combine(p.proj, rb0, 1.0, p.proj, Z, ly.mp, k, ycol(k), -1.0, tm, g.m(),
                                  part, count, &dst->res, dst, k, s, csnap));
            else
                CK(launch_combine(p.proj, nullptr, 0.0, p.basis, V, ly.ldv, k + 1, rho, 1.0, tm,
                                  g.m(), part, count, &dst->res, dst, k, s, csnap));
            if (ncp_stop) CK(launch_ncp(g, p.proj, tm, ncp, dst, k, s, snap));
        }
        CK(hipEventRecord(hr.ev[k % kRing], s));
        return ABG_OK;
    }

    int wait_step(int k, DevState &out)
    {
        CK(hipEventSynchronize(hr.ev[k % kRing]));
        out = hr.slots[k];
        return ABG_OK;
    }

    int sync_read(DevState &out)
    {
        CK(hipMemcpyAsync(&hr.slots[0], dst, sizeof(DevState), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        out = hr.slots[0];
        return ABG_OK;
    }

    // x = x0 + W[0..kk) c (BA)  or  x = x0 + B (W[0..kk) c)  (AB)
    int build_x(const double *c, int kk, const void *x0, void *x)
    {
        if (method == ABG_METHOD_BA) {
            CK(launch_combine(p.proj, x0, x0 ? 1.0 : 0.0, p.basis, V, ly.ldv, kk, c, 1.0, x,
                              g.n(), nullptr, nullptr, nullptr, nullptr, 0, s));
        } else {
            CK(launch_combine(p.proj, nullptr, 0.0, p.basis, V, ly.ldv, kk, c, 1.0, tm, g.m(),
                              nullptr, nullptr, nullptr, nullptr, 0, s));
            RC(back(tm, x));
            if (x0) CK(launch_axpy_inplace(p.proj, x, x0, g.n(), s));
        }
        return ABG_OK;
    }

    // ||b - A x|| into *out (default dst->res; uses tm); caller synchronises
    int literal_residual(const void *b, const void *x, double *out = nullptr)
    {
        RC(fwd(x, tm));
        int nb = 0;
        CK(launch_sub_norm(p.proj, b, tm, tm, g.m(), part, &nb, s));
        CK(launch_reduce_sqrt(part, nb, out ? out : &dst->res, s));
        return ABG_OK;
    }

    // Initialisation without a host synchronisation: scratch cleared, b - A x0,
    // r0 = (B)(b - A x0), and MGS step 0 (beta = ||r0|| into dst->hnext and g[0], w_1).
    // init: the solve's initial scalars (null: the caller owns *dst)
    int init_async(const void *b, const void *x0, const DevState *init)
    {
        const long long m = g.m();
        // one launch: the scalars, empty reduction slots, zeroed counters, H and g, the
        // forward projector's scratch (its padding must read zero), and the padding of the
        // MGS input vectors and of w_1 (a later step may read w_1 over a longer register
        // tile than step 0 writes); with x0 = 0, rb0 = b (zero-padded)
        const unsigned long long empty = slot_empty_bits();
        auto words = [](size_t bytes) { return (unsigned long long)(bytes / 4); };
        const FillRange fr[] = {
            {mgs_part, nullptr, 2ull * ly.mgs_cap, 0, (unsigned)empty, (unsigned)(empty >> 32)},
            {tick, nullptr, (unsigned long long)ld + 2, 0, 0u, 0u},
            {count, nullptr, 16, 0, 0u, 0u},
            {H, nullptr, 2ull * ld * k_max, 0, 0u, 0u},
            {gv, nullptr, 2ull * ld, 0, 0u, 0u},
            {fpws, nullptr, words(fp_workspace_bytes(g, p.proj)), 0, 0u, 0u},
            {q, nullptr, words(ly.ldv * sX), 0, 0u, 0u},
            {rb0, x0 ? nullptr : b, words(ly.mp * sX), x0 ? 0ull : words(m * sX), 0u, 0u},
            {V, nullptr, words(ly.ldv * dtype_size(p.basis)), 0, 0u, 0u},
        };
        CK(launch_init_fill(fr, (int)(sizeof fr / sizeof fr[0]), init, dst, s));
        if (x0) {
            RC(fwd(x0, tm));
            int nb = 0;
            CK(launch_sub_norm(p.proj, b, tm, rb0, m, part, &nb, s));
        }
        const void *r0 = rb0;
        if (method == ABG_METHOD_BA) {
            RC(back(rb0, q));
            r0 = q;
        }
        MgsLaunch M0 = mgs_args(r0, 0);
        M0.set_beta = init != nullptr;
        CK(launch_mgs(M0, s));
        return ABG_OK;
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

InstanceView instance_view(const Geometry &g, int method, int k_max, abg_precision p,
                           abg_stop st, void *ws)
{
    const Layout ly = make_layout(g, method, k_max, p, st);
    char *W = static_cast<char *>(ws);
    InstanceView v;
    v.V = W + ly.V;
    v.Z = ly.Z ? W + ly.Z : nullptr;
    v.cur = W + ly.cur;
    v.q = W + ly.q;
    v.rb0 = W + ly.rb0;
    v.tm = W + ly.tm;
    v.tn = W + ly.tn;
    v.fpws = W + ly.fpws;
    v.H = reinterpret_cast<double *>(W + ly.H);
    v.R = reinterpret_cast<double *>(W + ly.R);
    v.cs = reinterpret_cast<double *>(W + ly.cs);
    v.sn = reinterpret_cast<double *>(W + ly.sn);
    v.g = reinterpret_cast<double *>(W + ly.g);
    v.Y = reinterpret_cast<double *>(W + ly.Y);
    v.rho = reinterpret_cast<double *>(W + ly.rho);
    v.part = reinterpret_cast<double *>(W + ly.part);
    v.mgs_part = reinterpret_cast<double *>(W + ly.mgs_part);
    v.q64 = ly.q64 ? reinterpret_cast<double *>(W + ly.q64) : nullptr;
    v.count = reinterpret_cast<unsigned *>(W + ly.count);
    v.L = ly.L;
    v.ldv = ly.ldv;
    v.mp = ly.mp;
    v.np = ly.np;
    v.part_cap = 2048;
    v.mgs_rows = ly.mgs_rows;
    v.mgs_part_cap = ly.mgs_cap;
    return v;
}

int instance_init(const Geometry &g, int method, int kind, int k_max, abg_stop st,
                  abg_precision p, void *ws, const void *b, const void *x0, DevState *dst,
                  hipStream_t s)
{
    Solve S(g, method, kind, k_max, st, p, s, ws);
    S.dst = dst;
    return S.init_async(b, x0, nullptr);
}

int instance_form_x(const Geometry &g, int method, int kind, int k_max, abg_stop st,
                    abg_precision p, void *ws, int k, const void *b, const void *x0, void *x,
                    DevState *dst, double *lit, hipStream_t s)
{
    Solve S(g, method, kind, k_max, st, p, s, ws);
    S.dst = dst;
    RC(S.build_x(k > 0 ? S.ycol(k) : S.Y, k, x0, x));
    return S.literal_residual(b, x, lit);
}

hipError_t GroupHold::acquire(const Solve &S)
{
    s = S.s;
    long long u = 0;
    hipError_t e = mgs_group_units(S.p.proj, S.p.basis, S.ly.L, S.q64 != nullptr, &u);
    if (e != hipSuccess) return e;
    device_group_budget().acquire(u);
    units = u;
    return hipSuccess;
}

int run_solver(const Geometry &g, int method, int kind, const void *b, const void *x0,
               void *x, int k_max, abg_stop st, abg_precision p, void *ws, size_t ws_bytes,
               abg_info *info, hipStream_t s)
{
    Solve S(g, method, kind, k_max, st, p, s, ws);
    if (ws_bytes < S.ly.total) return ABG_ENOMEM;
    CK(S.lease.acquire(k_max, s));
    // the Gram-Schmidt groups must fit beside those of solves on other streams
    GroupHold hold;
    CK(hold.acquire(S));
    // launches of steps enqueued past the stop are left out of the launch timing
    struct ProfSolve {
        int last = 0;
        bool done = false;
        ProfSolve() { profile_solve_begin(); }
        void finish()
        {
            if (!done) profile_solve_end(last);
            done = true;
        }
        ~ProfSolve() { finish(); }
    } prof;
    const long long n = g.n();
    const double thr = st.kind == ABG_STOP_DP ? st.tau * st.noise_norm : 0.0;
    int k_stop = 0, k_done = 0, status = ABG_OK, n_literal = 0;
    double res_final = 0.0, ncp_final = 0.0;
    auto hist = [&](double *arr, int k, double v) {
        if (info && arr && k - 1 < info->hist_len) arr[k - 1] = v;
    };

    // device scalars: zero, with the DP candidate threshold
    DevState init{};
    init.dp_thr = st.kind == ABG_STOP_DP ? thr * (1.0 + dp_slack(p.basis)) : 0.0;

    // b - A x0, r0 = (B)(b - A x0), beta = ||r0|| into g[0], w_1; the host learns beta
    // (and a zero right-hand side or a NaN) from the scalars of step 1
    RC(S.init_async(b, x0, &init));
    DevState hs;
    bool zero_rhs = false;
    {
        double ncp_best = INFINITY, ncp_prev = 0.0;
        int best_k = 0;
        int k_sel = 0;        // step whose iterate is returned
        bool x_built = false; // x already holds x_{k_sel}, and res_final its residual
        // BA-GMRES with the NCP rule: ||r_k|| of the residual each step forms for the rule,
        // r_k = b - A x_0 - sum_i y_i (A w_i) from the stored products A w_i and the
        // coefficients x_k is built from (b - A x_k up to the rounding of the sum)
        const bool res_from_steps = method == ABG_METHOD_BA && st.kind == ABG_STOP_NCP;
        std::vector<double> res_k(res_from_steps ? k_max + 1 : 0, 0.0);
        RC(S.enqueue_step(1));
        for (int k = 1; k <= k_max && k_sel == 0; ++k) {
            if (k < k_max) RC(S.enqueue_step(k + 1));
            DevState sk;
            RC(S.wait_step(k, sk));
            if (sk.error & 1) return ABG_EDEVICE;
            if (sk.error) return ABG_ENAN;
            if (k == 1) {
                if (info) info->beta = sk.beta;
                if (sk.stop && sk.stop_reason == kStopZero) {
                    zero_rhs = true;
                    break;
                }
            }
            k_done = k;
            prof.last = k;
            hist(info ? info->ls_hist : nullptr, k, sk.ls);
            const bool stop_here = sk.stop && sk.stop_k == k;
            if (st.kind == ABG_STOP_DP) {
                double rk = sk.res;
                if (stop_here) {
                    // candidate: confirm with the explicit residual of x_k
                    RC(S.build_x(S.ycol(k), k, x0, x));
                    RC(S.literal_residual(b, x));
                    DevState h2;
                    RC(S.sync_read(h2));
                    ++n_literal;
                    rk = h2.res;
                    if (rk <= thr) {
                        k_sel = k;
                        x_built = true;
                        res_final = rk;
                    } else {
                        // rejected: resume; step k+1 was skipped, run it again
                        CK(launch_clear_stop(S.dst, s));
                        if (k < k_max) {
                            profile_drop_step(k + 1);
                            RC(S.enqueue_step(k + 1));
                        }
                    }
                }
                hist(info ? info->res_hist : nullptr, k, rk);
            } else if (st.kind == ABG_STOP_NCP) {
                hist(info ? info->res_hist : nullptr, k, sk.res);
                if (res_from_steps) res_k[k] = sk.res;
                hist(info ? info->ncp_hist : nullptr, k, sk.ncp);
                if (stop_here) {
                    k_sel = k - 1;   // d_k > d_{k-1}: x_{k-1} was closest to white noise
                    ncp_final = ncp_prev;
                    break;
                }
                if (sk.ncp < ncp_best) {
                    ncp_best = sk.ncp;
                    best_k = k;
                }
                ncp_prev = sk.ncp;
            }
            if (k_sel) break;
            if (sk.bd_k == k) {
                k_sel = k;
                status = ABG_BREAKDOWN;
                break;
            }
            if (k == k_max) {
                if (st.kind == ABG_STOP_NCP) {
                    k_sel = best_k;
                    ncp_final = ncp_best;
                } else {
                    k_sel = k;
                    status = st.kind == ABG_STOP_DP ? ABG_NOT_CONVERGED : ABG_OK;
                }
            }
        }
        if (zero_rhs) {
            if (x0) CK(hipMemcpyAsync(x, x0, (size_t)n * S.sX, hipMemcpyDeviceToDevice, s));
            else CK(launch_combine(p.proj, nullptr, 0.0, p.basis, S.V, S.ly.ldv, 0, S.Y, 1.0, x, n,
                                   nullptr, nullptr, nullptr, nullptr, 0, s));
            RC(S.literal_residual(b, x));
            RC(S.sync_read(hs));
            res_final = hs.res;
            status = ABG_ZERO_RHS;
            k_done = 0;
            prof.last = 0;
        } else {
            k_stop = k_sel;
            if (!x_built) {
                RC(S.build_x(S.ycol(k_sel), k_sel, x0, x));
                if (res_from_steps) {
                    // the returned iterate's residual was formed at its own step
                    res_final = res_k[k_sel];
                } else {
                    // explicit residual of the returned iterate (a DP-confirmed iterate
                    // has it already); a NaN/Inf anywhere in b shows here
                    RC(S.literal_residual(b, x));
                    RC(S.sync_read(hs));
                    res_final = hs.res;
                }
            }
            if (!std::isfinite(res_final)) return ABG_ENAN;
        }
    }

    if (info) {
        info->k_stop = k_stop;
        info->k_done = k_done;
        info->status = status;
        info->n_literal = n_literal;
        info->res_norm = res_final;
        info->ncp_dist = ncp_final;
        if (info->H && k_done > 0) {
            CK(hipMemcpyAsync(info->H, S.H, (size_t)S.ld * k_max * 8, hipMemcpyDeviceToHost, s));
            CK(hipStreamSynchronize(s));
        }
    }
    prof.finish();
    return status;
}

int gmres_error_history(const Geometry &g, int method, int kind, int k_max, abg_stop st,
                        abg_precision p, void *ws, size_t ws_bytes, const void *x0,
                        const void *x_ref, int k_done, double *err, hipStream_t s)
{
    Solve S(g, method, kind, k_max, st, p, s, ws);
    if (ws_bytes < S.ly.total) return ABG_ENOMEM;
    if (k_done < 0 || k_done > k_max) return ABG_EINVAL;
    CK(S.lease.acquire(k_max, s));
    // the workspace must hold k_done completed steps (their small-problem solutions)
    DevState h;
    RC(S.sync_read(h));
    if (h.k < k_done) return ABG_EINVAL;
    const long long n = g.n();
    for (int k = 1; k <= k_done; ++k) {
        // x_k into tn, then ||x_k - x_ref|| into host slot k
        RC(S.build_x(S.ycol(k), k, x0, S.tn));
        int nb = 0;
        CK(launch_sub_norm(p.proj, x_ref, S.tn, S.tn, n, S.part, &nb, s));
        CK(launch_reduce_sqrt(S.part, nb, &S.hr.dslots[k].err, s));
    }
    CK(hipStreamSynchronize(s));
    for (int k = 1; k <= k_done; ++k) err[k - 1] = S.hr.slots[k].err;
    return ABG_OK;
}

// ---- LSQR / LSMR -----------------------------------------------------------------------

namespace {

struct LsqLayout {
    size_t u, t, tres, ah, ahbar, r, v, sv, w, hbar, xprev, fpws, ncp, part, count, S, st, total;
};

LsqLayout make_lsq_layout(const Geometry &g, int method, int dtype)
{
    LsqLayout ly{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(std::max<size_t>(bytes, 1));
        return o;
    };
    const size_t sx = dtype_size(dtype);
    const size_t m = (size_t)g.m(), n = (size_t)g.n();
    const bool lsmr = method == ABG_METHOD_LSMR;
    ly.u = take(m * sx);
    ly.t = take(m * sx);
    ly.tres = take(m * sx);
    ly.ah = lsmr ? take(m * sx) : 0;
    ly.ahbar = lsmr ? take(m * sx) : 0;
    ly.r = lsmr ? take(m * sx) : 0;
    ly.v = take(n * sx);
    ly.sv = take(n * sx);
    ly.w = take(n * sx);               // LSQR w, LSMR h
    ly.hbar = lsmr ? take(n * sx) : 0;
    ly.xprev = take(n * sx);           // NCP runs: x_{k-1}
    ly.fpws = take(fp_workspace_bytes(g, dtype));
    ly.ncp = g.n_det >= 2 ? take(ncp_scratch_bytes(g)) : 0;
    ly.part = take(2048 * 8);
    ly.count = take(64);
    ly.S = take(sizeof(LsqScalars));
    ly.st = take(sizeof(DevState));
    ly.total = off;
    return ly;
}

}  // namespace

size_t lsq_workspace_bytes(const Geometry &g, int method, int dtype)
{
    return make_lsq_layout(g, method, dtype).total;
}

int run_lsq(const Geometry &g, int method, const void *b, const void *x0, void *x, int k_max,
            abg_stop st, int dtype, void *ws, size_t ws_bytes, abg_info *info,
            const void *x_ref, double *err_hist, hipStream_t s)
{
    const LsqLayout ly = make_lsq_layout(g, method, dtype);
    if (ws_bytes < ly.total) return ABG_ENOMEM;
    const bool lsmr = method == ABG_METHOD_LSMR;
    char *W = static_cast<char *>(ws);
    void *u = W + ly.u, *t = W + ly.t, *tres = W + ly.tres, *v = W + ly.v, *sv = W + ly.sv,
         *w = W + ly.w, *fpws = W + ly.fpws;
    void *ah = lsmr ? W + ly.ah : nullptr, *ahbar = lsmr ? W + ly.ahbar : nullptr;
    void *r = lsmr ? W + ly.r : nullptr, *hbar = lsmr ? W + ly.hbar : nullptr;
    const bool ncp_stop = st.kind == ABG_STOP_NCP;
    if (ncp_stop && !ly.ncp) return ABG_EINVAL;
    void *xprev = ncp_stop ? W + ly.xprev : nullptr;
    double *ncp = ncp_stop ? reinterpret_cast<double *>(W + ly.ncp) : nullptr;
    double *part = reinterpret_cast<double *>(W + ly.part);
    unsigned *count = reinterpret_cast<unsigned *>(W + ly.count);
    LsqScalars *S = reinterpret_cast<LsqScalars *>(W + ly.S);
    DevState *dst = reinterpret_cast<DevState *>(W + ly.st);
    const long long m = g.m(), n = g.n();
    const size_t sx = dtype_size(dtype);
    // the forward projector's exact transpose
    const int bkind = g.model == ABG_FP_STRIP    ? ABG_BP_STRIP_T
                      : g.model == ABG_FP_JOSEPH ? ABG_BP_JOSEPH_T
                                                 : ABG_BP_ADJ;
    HostLease lease;
    CK(lease.acquire(k_max, s));
    HostRes &hr = lease.r;
    struct ProfSolve {
        int last = 0;
        bool done = false;
        ProfSolve() { profile_solve_begin(); }
        void finish()
        {
            if (!done) profile_solve_end(last);
            done = true;
        }
        ~ProfSolve() { finish(); }
    } prof;
    const double thr = st.kind == ABG_STOP_DP ? st.tau * st.noise_norm : 0.0;
    DevState init{};
    init.dp_thr = st.kind == ABG_STOP_DP ? thr * (1.0 + dp_slack(dtype)) : 0.0;

    // scalars: alpha_0 = 0, beta_0 = 1 (the first u step copies t), rho_0 = 1
    auto words = [](size_t bytes) { return (unsigned long long)(bytes / 4); };
    const unsigned one_hi = 0x3ff00000u;
    const size_t xb = (size_t)n * sx;
    std::vector<FillRange> fr = {
        {count, nullptr, 16, 0, 0u, 0u},
        {S, nullptr, words(sizeof(LsqScalars)), 0, 0u, 0u},
        {u, nullptr, words((size_t)m * sx), 0, 0u, 0u},  // the first step reads 0 * u
        {v, nullptr, words(xb), 0, 0u, 0u},
        {fpws, nullptr, words(fp_workspace_bytes(g, dtype)), 0, 0u, 0u},
        {x, x0, words(xb), x0 ? words(xb) : 0, 0u, 0u},
    };
    if (!x0) fr.push_back({t, b, words((size_t)m * sx), words((size_t)m * sx), 0u, 0u});
    if (lsmr) {
        fr.push_back({ah, nullptr, words((size_t)m * sx), 0, 0u, 0u});
        fr.push_back({ahbar, nullptr, words((size_t)m * sx), 0, 0u, 0u});
        if (!x0) fr.push_back({r, b, words((size_t)m * sx), words((size_t)m * sx), 0u, 0u});
    }
    CK(launch_init_fill(fr.data(), (int)fr.size(), &init, dst, s));
    {
        // beta_0 = 1 and rho_0 = 1 (after the zero fill of the scalars)
        const FillRange ones[] = {
            {&S->beta, nullptr, 2, 0, 0u, one_hi},
            {&S->rho_prev, nullptr, 2, 0, 0u, one_hi},
            {&S->rhobar_prev, nullptr, 2, 0, 0u, one_hi},
            {&S->cbar, nullptr, 2, 0, 0u, one_hi},
        };
        CK(launch_init_fill(ones, 4, nullptr, nullptr, s));
    }
    if (x0) {
        CK(launch_forward(g, dtype, x0, t, fpws, s, nullptr, 0, true));
        int nb = 0;
        CK(launch_sub_norm(dtype, b, t, t, m, part, &nb, s));
        if (lsmr) CK(hipMemcpyAsync(r, t, (size_t)m * sx, hipMemcpyDeviceToDevice, s));
    }
    // beta_1 u_1 = b - A x0, alpha_1 v_1 = A^T u_1, v_1, w_1 / h_1 and the scalars
    CK(launch_lsq_u(dtype, u, t, ah, m, S, part, count, nullptr, 0, s));
    CK(launch_back(g, bkind, dtype, u, sv, s));
    CK(launch_lsq_v(dtype, v, sv, n, S, part, count, nullptr, 0, s));
    CK(launch_lsq_start(dtype, v, w, hbar, n, S, count, dst, lsmr ? 1 : 0, s));

    auto enqueue_step = [&](int k) -> int {
        CK(launch_forward(g, dtype, v, t, fpws, s, dst, k, true));
        CK(launch_lsq_u(dtype, u, t, ah, m, S, part, count, dst, k, s));
        CK(launch_back(g, bkind, dtype, u, sv, s, dst, k));
        CK(launch_lsq_v(dtype, v, sv, n, S, part, count, dst, k, s));
        // the scalars go to host slot k from the step's last kernel
        DevState *snap = ncp_stop ? nullptr : hr.dslots + k;
        if (lsmr) {
            CK(launch_lsmr_x(dtype, x, xprev, w, hbar, v, n, S, count, dst, k, s));
            CK(launch_lsmr_r(dtype, ah, ahbar, r, m, S, part, count, dst, k, snap, s));
        } else {
            CK(launch_lsqr_x(dtype, x, xprev, w, v, n, S, count, dst, k, snap, s));
        }
        if (ncp_stop) {
            // the NCP distance of the explicit residual b - A x_k (its norm into res)
            CK(launch_forward(g, dtype, x, tres, fpws, s, dst, k, true));
            int nb = 0;
            CK(launch_sub_norm(dtype, b, tres, tres, m, part, &nb, s));
            CK(launch_reduce_sqrt(part, nb, &dst->res, s));
            CK(launch_ncp(g, dtype, tres, ncp, dst, k, s, hr.dslots + k));
        }
        if (x_ref) {
            // ||x_k - x_ref|| into slot k, after the step's copy of the scalars (sv is
            // free until the next step's back projection)
            int nb = 0;
            CK(launch_sub_norm(dtype, x_ref, x, sv, n, part, &nb, s));
            CK(launch_reduce_sqrt(part, nb, &hr.dslots[k].err, s));
        }
        CK(hipEventRecord(hr.ev[k % kRing], s));
        return ABG_OK;
    };
    auto sync_read = [&](DevState &out) -> int {
        CK(hipMemcpyAsync(&hr.slots[0], dst, sizeof(DevState), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        out = hr.slots[0];
        return ABG_OK;
    };
    // ||b - A x|| into dst->res
    auto literal_residual = [&]() -> int {
        CK(launch_forward(g, dtype, x, tres, fpws, s, nullptr, 0, true));
        int nb = 0;
        CK(launch_sub_norm(dtype, b, tres, tres, m, part, &nb, s));
        CK(launch_reduce_sqrt(part, nb, &dst->res, s));
        return ABG_OK;
    };
    auto hist = [&](double *arr, int k, double val) {
        if (info && arr && k - 1 < info->hist_len) arr[k - 1] = val;
    };

    int k_sel = -1, k_done = 0, status = ABG_OK, n_literal = 0;
    double res_final = 0.0, ncp_prev = 0.0, ncp_final = 0.0;
    bool res_known = false, from_prev = false;
    RC(enqueue_step(1));
    for (int k = 1; k <= k_max && k_sel < 0; ++k) {
        if (k < k_max) RC(enqueue_step(k + 1));
        CK(hipEventSynchronize(hr.ev[k % kRing]));
        const DevState sk = hr.slots[k];
        if (sk.error & 1) return ABG_EDEVICE;
        if (sk.error) return ABG_ENAN;
        if (k == 1) {
            if (info) info->beta = sk.beta;
            if (sk.stop && sk.stop_reason == kStopZero) {
                // b - A x0 = 0, or A^T (b - A x0) = 0: x0 is returned
                status = sk.beta == 0.0 ? ABG_ZERO_RHS : ABG_BREAKDOWN;
                k_sel = 0;
                break;
            }
        }
        k_done = k;
        prof.last = k;
        hist(info ? info->res_hist : nullptr, k, sk.res);
        hist(info ? info->ls_hist : nullptr, k, sk.ls);
        if (x_ref) err_hist[k - 1] = sk.err;
        if (ncp_stop) {
            hist(info ? info->ncp_hist : nullptr, k, sk.ncp);
            if (sk.stop && sk.stop_k == k) {
                // d_k > d_{k-1}: x_{k-1} (kept by the step's x kernel) is returned
                k_sel = k - 1;
                ncp_final = ncp_prev;
                from_prev = true;
                break;
            }
            ncp_prev = sk.ncp;
            ncp_final = sk.ncp;
        }
        if (st.kind == ABG_STOP_DP && sk.stop && sk.stop_k == k) {
            // candidate: confirm with the explicit residual of x_k (later steps are halted)
            RC(literal_residual());
            DevState h2;
            RC(sync_read(h2));
            ++n_literal;
            if (h2.res <= thr) {
                k_sel = k;
                res_final = h2.res;
                res_known = true;
                break;
            }
            CK(launch_clear_stop(dst, s));
            if (k < k_max) {
                profile_drop_step(k + 1);
                RC(enqueue_step(k + 1));
            }
        }
        if (sk.bd_k == k) {
            k_sel = k;
            status = ABG_BREAKDOWN;
            break;
        }
        if (k == k_max) {
            k_sel = k;
            status = st.kind == ABG_STOP_DP ? ABG_NOT_CONVERGED : ABG_OK;
        }
    }
    if (k_sel < 0) k_sel = k_done;
    if (from_prev) CK(hipMemcpyAsync(x, xprev, (size_t)n * sx, hipMemcpyDeviceToDevice, s));
    if (!res_known) {
        RC(literal_residual());
        DevState hs;
        RC(sync_read(hs));
        res_final = hs.res;
    }
    if (!std::isfinite(res_final)) return ABG_ENAN;
    if (status == ABG_ZERO_RHS || (k_sel == 0 && status == ABG_BREAKDOWN)) k_done = 0;
    if (info) {
        info->k_stop = k_sel;
        info->k_done = k_done;
        info->status = status;
        info->n_literal = n_literal;
        info->res_norm = res_final;
        info->ncp_dist = ncp_stop ? ncp_final : 0.0;
    }
    prof.finish();
    return status;
}

}  // namespace abg
