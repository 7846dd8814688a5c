// Host runtime behind the C ABI of include/fas.h: object lifetimes,
// parameter checks, the smoother stage loop, the FAS recursion and dual
// time stepping, all enqueued on the caller's HIP stream.
#include "fas.h"
#include "fas_internal.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace fas;

namespace {

thread_local std::string g_err = "no error";

fas_status fail(fas_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(e_ == hipErrorOutOfMemory ? FAS_ENOMEM : FAS_EDEVICE,                 \
                        std::string(#call) + ": " + hipGetErrorString(e_));                   \
    } while (0)

#define STCHK(expr)                                   \
    do {                                              \
        fas_status s_ = (expr);                       \
        if (s_ != FAS_OK) return s_;                  \
    } while (0)

// Table "RK smoothers": alpha; beta of ARK3J for the 3-stage schemes and of
// ARK5J for every 5-stage scheme; W (additive W) or P ~ J (preconditioned ARK).
struct Scheme {
    int s;
    double alpha[5], beta[5];
    int aw;
};
const Scheme SCHEMES[6] = {
    {3, {0.1481, 2.0 / 5.0, 1.0}, {1.0, 0.5, 0.5}, 1},
    {3, {0.1481, 2.0 / 5.0, 1.0}, {1.0, 0.5, 0.5}, 0},
    {5, {1.0 / 4.0, 1.0 / 6.0, 3.0 / 8.0, 1.0 / 2.0, 1.0}, {1.0, 0.0, 0.56, 0.0, 0.44}, 1},
    {5, {0.0533, 0.1263, 0.2375, 0.4414, 1.0}, {1.0, 0.0, 0.56, 0.0, 0.44}, 1},
    {5, {0.0695, 0.1602, 0.2898, 0.5060, 1.0}, {1.0, 0.0, 0.56, 0.0, 0.44}, 1},
    {5, {0.0533, 0.1263, 0.2375, 0.4414, 1.0}, {1.0, 0.0, 0.56, 0.0, 0.44}, 0},
};

Lay make_lay(int ni, int nj, int nw, int topo) {
    Lay L;
    L.ni = ni;
    L.nj = nj;
    L.NI = ni + 2 * NG;
    L.NJ = nj + 2 * NG;
    L.NS = (L.NI + L.NJ - 1) * L.NJ;
    L.nw = topo == FAS_CGRID ? nw : 0;
    L.topo = topo;
    return L;
}

}  // namespace

struct fas_grid_s {
    int topo, ni, nj, nw, nlev, device;
    std::vector<Lay> lay;
    std::vector<double *> geo, xn, yn;
};

struct fas_state_s {
    fas_grid g;
    fas_params p;
    hipStream_t st;
    int nlev;
    Phys ph;
    Scheme sc;
    std::vector<LevelDev> lv;
    std::vector<int> has_src;
    int n_cycles = 0;
    int bdf = 0;
    int have_un = 0;
    double dt = 0.0;
    double *d_norm = nullptr;   // device scalar
    std::vector<void *> allocs;
    // optional per-kernel-class timing with HIP events on the state's stream
    int prof = 0;
    struct Rec { int cls; hipEvent_t a, b; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    double prof_ms[FAS_PROF_NCLASS] = {0};
    int64_t prof_n[FAS_PROF_NCLASS] = {0};
};

// --------------------------------------------------------------------- grid
extern "C" void fas_params_default(fas_params *p) {
    std::memset(p, 0, sizeof(*p));
    p->version = FAS_PARAMS_VERSION;
    p->model = FAS_EULER;
    p->scheme = FAS_AW3;
    p->n_ramp = 2;
    p->eta = 0.5;
    p->d_cut = 0.5;
    p->cfl = 1.0e4;
    p->cfl_ramp = 20.0;
    p->ramp_growth = 1.0;
    p->kappa2c = 0.125;
    p->mach = 0.8;
    p->alpha_deg = 0.0;
    p->reynolds = 1.0e7;
    p->prandtl = 0.75;
    p->prandtl_t = 0.9;
    p->n_levels = 1;
    p->cycle_gamma = 1;
    p->nu1 = 1;
    p->precond_fp32 = 0;
}

extern "C" fas_status fas_grid_create(int32_t topology, int32_t ni, int32_t nj, int32_t n_wake,
                                      const double *x_nodes, const double *y_nodes,
                                      int32_t n_levels, fas_grid *out) {
    if (!out || !x_nodes || !y_nodes) return fail(FAS_EINVAL, "null argument");
    *out = nullptr;
    if (topology != FAS_BOX && topology != FAS_CGRID) return fail(FAS_EINVAL, "bad topology");
    if (n_levels < 1 || n_levels > 8) return fail(FAS_EINVAL, "n_levels must be in [1, 8]");
    const int f = 1 << (n_levels - 1);
    if (ni < 4 || nj < 4 || ni % f || nj % f) return fail(FAS_EINVAL, "ni, nj must be >= 4 and divisible by 2^(n_levels-1)");
    if (nj > 512) return fail(FAS_EINVAL, "nj must be <= 512 (one sweep row per thread)");
    if (topology == FAS_CGRID) {
        if (n_wake < 1 || 2 * n_wake >= ni || n_wake % f)
            return fail(FAS_EINVAL, "n_wake must be in [1, ni/2) and divisible by 2^(n_levels-1)");
        if ((ni / f) < 4 || (nj / f) < 2) return fail(FAS_EINVAL, "coarsest level too small");
    }
    fas_grid g = new fas_grid_s();
    g->topo = topology;
    g->ni = ni;
    g->nj = nj;
    g->nw = topology == FAS_CGRID ? n_wake : 0;
    g->nlev = n_levels;
    (void)hipGetDevice(&g->device);
    auto cleanup = [&](fas_status s) {
        fas_grid_destroy(g);
        return s;
    };
    const int W = ni + 1;
    for (int l = 0; l < n_levels; ++l) {
        int s = 1 << l;
        int nil = ni / s, njl = nj / s;
        Lay L = make_lay(nil, njl, g->nw / s, topology);
        g->lay.push_back(L);
        std::vector<double> hx((size_t)(nil + 1) * (njl + 1)), hy(hx.size());
        for (int J = 0; J <= njl; ++J)
            for (int I = 0; I <= nil; ++I) {
                hx[(size_t)J * (nil + 1) + I] = x_nodes[(size_t)(J * s) * W + I * s];
                hy[(size_t)J * (nil + 1) + I] = y_nodes[(size_t)(J * s) * W + I * s];
            }
        double *dx = nullptr, *dy = nullptr, *geo = nullptr;
        if (hipMalloc(&dx, hx.size() * sizeof(double)) != hipSuccess ||
            hipMalloc(&dy, hy.size() * sizeof(double)) != hipSuccess ||
            hipMalloc(&geo, (size_t)G_NPLANES * L.NS * sizeof(double)) != hipSuccess) {
            if (dx) g->xn.push_back(dx);
            if (dy) g->yn.push_back(dy);
            if (geo) g->geo.push_back(geo);
            return cleanup(fail(FAS_ENOMEM, "grid allocation failed"));
        }
        g->xn.push_back(dx);
        g->yn.push_back(dy);
        g->geo.push_back(geo);
        if (hipMemcpy(dx, hx.data(), hx.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(dy, hy.data(), hy.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemset(geo, 0, (size_t)G_NPLANES * L.NS * sizeof(double)) != hipSuccess)
            return cleanup(fail(FAS_EDEVICE, "grid upload failed"));
        if (l == 0) launch_geom_interior(L, dx, dy, geo, nullptr, nullptr, nullptr, 0);
        else launch_geom_interior(L, dx, dy, geo, nullptr, &g->lay[l - 1], g->geo[l - 1], 0);
        launch_geom_ghost(L, dx, dy, geo, 0);
    }
    if (hipDeviceSynchronize() != hipSuccess) return cleanup(fail(FAS_EDEVICE, "geometry kernels failed"));
    // every volume must be positive (right-handed grid)
    {
        const Lay &L = g->lay[0];
        std::vector<double> vol(L.NS);
        if (hipMemcpy(vol.data(), g->geo[0] + (size_t)G_VOL * L.NS, L.NS * sizeof(double),
                      hipMemcpyDeviceToHost) != hipSuccess)
            return cleanup(fail(FAS_EDEVICE, "volume check failed"));
        for (int j = 0; j < nj; ++j)
            for (int i = 0; i < ni; ++i)
                if (!(vol[L.slot(i, j)] > 0.0))
                    return cleanup(fail(FAS_EINVAL, "non-positive cell volume (grid must be right-handed)"));
    }
    *out = g;
    return FAS_OK;
}

extern "C" void fas_grid_destroy(fas_grid g) {
    if (!g) return;
    for (auto p : g->geo) (void)hipFree(p);
    for (auto p : g->xn) (void)hipFree(p);
    for (auto p : g->yn) (void)hipFree(p);
    delete g;
}

// -------------------------------------------------------------------- state
static fas_status check_params(const fas_params *p, int grid_levels) {
    if (!p || p->version != FAS_PARAMS_VERSION) return fail(FAS_EINVAL, "fas_params version mismatch");
    if (p->model != FAS_EULER && p->model != FAS_RANS_BL) return fail(FAS_EINVAL, "bad model");
    if (p->scheme < 0 || p->scheme > 5) return fail(FAS_EINVAL, "bad scheme");
    if (p->n_levels < 1 || p->n_levels > grid_levels) return fail(FAS_EINVAL, "n_levels exceeds the grid's levels");
    if (p->cycle_gamma < 1 || p->cycle_gamma > 2 || p->nu1 < 1) return fail(FAS_EINVAL, "bad cycle parameters");
    if (!(p->cfl > 0.0) || !(p->cfl_ramp > 0.0) || !(p->eta > 0.0) || p->d_cut < 0.0 || p->d_cut > 1.0)
        return fail(FAS_EINVAL, "bad smoother parameters");
    if (!(p->mach > 0.0) || (p->model == FAS_RANS_BL && !(p->reynolds > 0.0)))
        return fail(FAS_EINVAL, "bad flow parameters");
    return FAS_OK;
}

static void set_phys(fas_state s) {
    const fas_params &p = s->p;
    Phys &ph = s->ph;
    ph.mach = p.mach;
    ph.alpha_deg = p.alpha_deg;
    ph.re = p.reynolds;
    ph.pr = p.prandtl;
    ph.prt = p.prandtl_t;
    ph.mu_inf = p.model == FAS_RANS_BL ? p.mach * std::sqrt(GAM) / p.reynolds : 0.0;
    double V = p.mach * std::sqrt(GAM);
    double a = p.alpha_deg * (M_PI / 180.0);
    double vx = V * std::cos(a), vy = V * std::sin(a);
    ph.uinf[0] = 1.0;
    ph.uinf[1] = vx;
    ph.uinf[2] = vy;
    ph.uinf[3] = 1.0 / (GAM - 1.0) + 0.5 * (vx * vx + vy * vy);
    ph.eta = p.eta;
    ph.d_cut = p.d_cut;
    ph.kappa2c = p.kappa2c;
    ph.rans = p.model == FAS_RANS_BL;
    s->sc = SCHEMES[p.scheme];
}

extern "C" void fas_state_destroy(fas_state s) {
    if (!s) return;
    if (s->st) (void)hipStreamSynchronize(s->st);
    for (auto &r : s->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : s->pool) (void)hipEventDestroy(e);
    for (auto p : s->allocs) (void)hipFree(p);
    delete s;
}

extern "C" fas_status fas_state_create(fas_grid g, const fas_params *p, const double *u0,
                                       void *stream, fas_state *out) {
    if (!g || !out || !u0) return fail(FAS_EINVAL, "null argument");
    *out = nullptr;
    STCHK(check_params(p, g->nlev));
    fas_state s = new fas_state_s();
    s->g = g;
    s->p = *p;
    s->st = (hipStream_t)stream;
    s->nlev = p->n_levels;
    set_phys(s);
    auto cleanup = [&](fas_status st) {
        fas_state_destroy(s);
        return st;
    };
    for (int l = 0; l < s->nlev; ++l) {
        LevelDev d;
        std::memset(&d, 0, sizeof(d));
        d.L = g->lay[l];
        d.geo = g->geo[l];
        const size_t NS = d.L.NS;
        const size_t nd = (size_t)(4 * 8 + 2 + Q_NPLANES + V_NPLANES) * NS + 256;
        const size_t nb = (size_t)BLK_NPLANES * NS * 8 + (size_t)8 * NS * 8;
        double *base = nullptr;
        char *bb = nullptr;
        if (hipMalloc(&base, nd * sizeof(double)) != hipSuccess) return cleanup(fail(FAS_ENOMEM, "state allocation failed"));
        s->allocs.push_back(base);
        if (hipMalloc(&bb, nb) != hipSuccess) return cleanup(fail(FAS_ENOMEM, "state allocation failed"));
        s->allocs.push_back(bb);
        if (hipMemsetAsync(base, 0, nd * sizeof(double), s->st) != hipSuccess ||
            hipMemsetAsync(bb, 0, nb, s->st) != hipSuccess)
            return cleanup(fail(FAS_EDEVICE, "state clear failed"));
        double *q = base;
        auto take = [&](size_t n) { double *r = q; q += n * NS; return r; };
        d.u = take(4); d.u0 = take(4); d.acc = take(4); d.F = take(4);
        d.src = take(4); d.ut = take(4); d.un = take(4); d.unm1 = take(4);
        d.dts = take(1); d.mut = take(1); d.cq = take(Q_NPLANES); d.vg = take(V_NPLANES);
        d.red = q;
        d.blk = bb;
        d.g = bb + (size_t)BLK_NPLANES * NS * 8;
        d.y = bb + (size_t)BLK_NPLANES * NS * 8 + (size_t)4 * NS * 8;
        s->lv.push_back(d);
    }
    s->has_src.assign(s->nlev, 0);
    if (hipMalloc(&s->d_norm, 8 * sizeof(double)) != hipSuccess) return cleanup(fail(FAS_ENOMEM, "allocation failed"));
    s->allocs.push_back(s->d_norm);
    launch_unpack(s->lv[0].L, u0, s->lv[0].u, 4, s->st);
    if (hipGetLastError() != hipSuccess) return cleanup(fail(FAS_EDEVICE, "kernel launch failed"));
    *out = s;
    return FAS_OK;
}

extern "C" fas_status fas_state_set_params(fas_state s, const fas_params *p) {
    if (!s) return fail(FAS_EINVAL, "null state");
    STCHK(check_params(p, s->g->nlev));
    if (p->n_levels != s->nlev) return fail(FAS_EINVAL, "n_levels cannot change after creation");
    s->p = *p;
    set_phys(s);
    return FAS_OK;
}

extern "C" fas_status fas_set_state(fas_state s, const double *u) {
    if (!s || !u) return fail(FAS_EINVAL, "null argument");
    launch_unpack(s->lv[0].L, u, s->lv[0].u, 4, s->st);
    HIPCHK(hipGetLastError());
    return FAS_OK;
}

extern "C" fas_status fas_get_state(fas_state s, double *u, double *mu_t) {
    if (!s) return fail(FAS_EINVAL, "null state");
    if (u) launch_pack(s->lv[0].L, s->lv[0].u, u, 4, s->st);
    if (mu_t) launch_pack(s->lv[0].L, s->lv[0].mut, mu_t, 1, s->st);
    HIPCHK(hipGetLastError());
    return FAS_OK;
}

extern "C" fas_status fas_get_level(fas_state s, int32_t level, double *u, double *source) {
    if (!s || level < 0 || level >= s->nlev) return fail(FAS_EINVAL, "bad level");
    const LevelDev &d = s->lv[level];
    if (u) launch_pack(d.L, d.u, u, 4, s->st);
    if (source) launch_pack(d.L, d.src, source, 4, s->st);
    HIPCHK(hipGetLastError());
    return FAS_OK;
}

// ----------------------------------------------------------- building blocks
namespace {

hipEvent_t take_event(fas_state s) {
    if (!s->pool.empty()) {
        hipEvent_t e = s->pool.back();
        s->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// brackets a launch with events when profiling is on
struct Prof {
    fas_state s;
    int cls;
    hipEvent_t a = nullptr;
    Prof(fas_state s_, int c) : s(s_), cls(c) {
        if (s->prof) {
            a = take_event(s);
            (void)hipEventRecord(a, s->st);
        }
    }
    ~Prof() {
        if (a) {
            hipEvent_t b = take_event(s);
            (void)hipEventRecord(b, s->st);
            s->recs.push_back({cls, a, b});
        }
    }
};

bool fine_rans(fas_state s, int l) { return l == 0 && s->p.model == FAS_RANS_BL; }

double tau_of(fas_state s) {
    if (s->bdf == 2) return 3.0 / (2.0 * s->dt);
    if (s->bdf == 1) return 1.0 / s->dt;
    return 0.0;
}

double cfl_now(fas_state s) {
    const fas_params &p = s->p;
    if (s->n_cycles < p.n_ramp) return std::fmin(p.cfl, p.cfl_ramp);
    if (p.ramp_growth > 1.0)
        return std::fmin(p.cfl, p.cfl_ramp * std::pow(p.ramp_growth, (double)(s->n_cycles - p.n_ramp + 1)));
    return p.cfl;
}

// ghosts, cell quantities, vertex gradients (fine RANS) and, on request,
// the Baldwin-Lomax eddy viscosity for the level's current solution
void prep(fas_state s, int l, bool with_bl) {
    LevelDev &d = s->lv[l];
    const int noslip = s->p.model == FAS_RANS_BL;
    launch_ghost_state(d.L, d.geo, d.u, s->ph, noslip, s->st);
    launch_cell_quantities(d.L, d.geo, d.u, d.cq, s->p.model == FAS_RANS_BL, s->st);
    if (fine_rans(s, l)) {
        launch_vertex_gradients(d.L, d.geo, d.u, d.cq, d.vg, s->st);
        if (with_bl) {
            launch_baldwin_lomax(d.L, d.geo, d.u, d.cq, d.vg, d.mut, s->ph, s->st);
            launch_mut_ghosts(d.L, d.mut, s->st);
        }
    }
}

ResArgs res_args(fas_state s, int l, int mode, int forcing) {
    ResArgs a;
    std::memset(&a, 0, sizeof(a));
    a.fine = l == 0;
    a.viscous = fine_rans(s, l);
    a.bdf = s->bdf;
    a.dt = s->dt;
    a.forcing = forcing && s->has_src[l];
    a.mode = mode;
    a.aw = s->sc.aw;
    a.fp32 = s->p.precond_fp32;
    return a;
}

// F_l(u_l) (- s_l) into lv[l].F, eddy viscosity evaluated at u_l
void eval_F(fas_state s, int l, bool forcing) {
    LevelDev &d = s->lv[l];
    prep(s, l, fine_rans(s, l));
    ResArgs a = res_args(s, l, 0, forcing);
    launch_residual(d.L, d.geo, d.u, d.cq, d.vg, d.mut, d.un, d.unm1, d.src, s->ph, a, d.F, d.acc,
                    d.dts, d.blk, d.g, s->st);
}

// frozen quantities of one smoother iteration: dt*, eddy viscosity, blocks
void prepare_iteration(fas_state s, int l, double cfl) {
    LevelDev &d = s->lv[l];
    prep(s, l, fine_rans(s, l));
    launch_local_time_step(d.L, d.geo, d.u, d.dts, cfl, s->st);
    Prof pr(s, FAS_PROF_BLOCKS);
    launch_blocks(d.L, d.geo, d.u, d.cq, d.mut, d.dts, s->ph, s->sc.aw, tau_of(s), fine_rans(s, l),
                  s->p.precond_fp32, d.blk, s->st);
}

// one smoother iteration (Section 4 low-storage stages)
void smooth_once(fas_state s, int l) {
    LevelDev &d = s->lv[l];
    launch_axpby_interior(d.L, 1.0, d.u, 0.0, nullptr, d.u0, 4, s->st);
    prepare_iteration(s, l, cfl_now(s));
    for (int k = 0; k < s->sc.s; ++k) {
        if (k > 0) prep(s, l, false);
        ResArgs a = res_args(s, l, 1, 1);
        a.stage = k;
        a.beta = s->sc.beta[k];
        {
            Prof pr(s, FAS_PROF_RESIDUAL);
            launch_residual(d.L, d.geo, d.u, d.cq, d.vg, d.mut, d.un, d.unm1, d.src, s->ph, a, d.F,
                            d.acc, d.dts, d.blk, d.g, s->st);
        }
        SweepArgs sw;
        sw.update = 1;
        sw.alpha = s->sc.alpha[k];
        sw.aw = s->sc.aw;
        sw.u = d.u;
        sw.u0 = d.u0;
        sw.dts = d.dts;
        sw.xout = nullptr;
        Prof pr(s, FAS_PROF_SWEEP);
        launch_sgs(d.L, d.blk, d.g, d.y, sw, s->p.precond_fp32, s->st);
    }
}

void cycle(fas_state s, int l) {
    const int nsm = l < s->nlev - 1 ? s->p.nu1 : 1;
    for (int k = 0; k < nsm; ++k) smooth_once(s, l);
    if (l == s->nlev - 1) return;
    LevelDev &f = s->lv[l], &c = s->lv[l + 1];
    eval_F(s, l, false);
    // r_l = s_l - F_l(u_l)
    if (s->has_src[l]) launch_axpby_interior(f.L, -1.0, f.F, 1.0, f.src, f.F, 4, s->st);
    else launch_axpby_interior(f.L, -1.0, f.F, 0.0, nullptr, f.F, 4, s->st);
    launch_restrict(f.L, c.L, f.geo, c.geo, f.u, c.u, c.ut, s->st);
    launch_restrict(f.L, c.L, f.geo, c.geo, f.F, c.acc, nullptr, s->st);
    s->has_src[l + 1] = 0;
    eval_F(s, l + 1, false);
    launch_axpby_interior(c.L, 1.0, c.F, 1.0, c.acc, c.src, 4, s->st);
    s->has_src[l + 1] = 1;
    for (int k = 0; k < s->p.cycle_gamma; ++k) cycle(s, l + 1);
    launch_prolong(f.L, c.L, c.u, c.ut, f.u, s->st);
}

fas_status norm(fas_state s, double *out) {
    eval_F(s, 0, false);
    LevelDev &d = s->lv[0];
    launch_norm(d.L, d.F, d.red, s->d_norm, s->st);
    HIPCHK(hipMemcpyAsync(out, s->d_norm, sizeof(double), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return FAS_OK;
}

}  // namespace

extern "C" fas_status fas_residual(fas_state s, int32_t level, double *F_out) {
    if (!s || !F_out || level < 0 || level >= s->nlev) return fail(FAS_EINVAL, "bad argument");
    eval_F(s, level, true);
    launch_pack(s->lv[level].L, s->lv[level].F, F_out, 4, s->st);
    HIPCHK(hipGetLastError());
    return FAS_OK;
}

extern "C" fas_status fas_smooth(fas_state s, int32_t level, int32_t n_iter) {
    if (!s || level < 0 || level >= s->nlev || n_iter < 0) return fail(FAS_EINVAL, "bad argument");
    for (int k = 0; k < n_iter; ++k) smooth_once(s, level);
    HIPCHK(hipGetLastError());
    return FAS_OK;
}

namespace fas {
void launch_dinv(const Lay &L, const void *blk, const double *r, void *g, int fp32, hipStream_t st);
}

extern "C" fas_status fas_sgs_apply(fas_state s, int32_t level, const double *r, double *x) {
    if (!s || !r || !x || level < 0 || level >= s->nlev) return fail(FAS_EINVAL, "bad argument");
    LevelDev &d = s->lv[level];
    prepare_iteration(s, level, cfl_now(s));
    launch_unpack(d.L, r, d.F, 4, s->st);
    launch_dinv(d.L, d.blk, d.F, d.g, s->p.precond_fp32, s->st);
    SweepArgs sw;
    std::memset(&sw, 0, sizeof(sw));
    sw.xout = d.acc;
    launch_sgs(d.L, d.blk, d.g, d.y, sw, s->p.precond_fp32, s->st);
    launch_pack(d.L, d.acc, x, 4, s->st);
    HIPCHK(hipGetLastError());
    return FAS_OK;
}

extern "C" fas_status fas_cycle(fas_state s, int32_t max_cycles, double drop_orders, double *res_hist,
                                int32_t *n_done) {
    if (!s || max_cycles < 0) return fail(FAS_EINVAL, "bad argument");
    double h0 = 0.0, h = 0.0;
    STCHK(norm(s, &h0));
    if (res_hist) res_hist[0] = h0;
    int done = 0;
    fas_status st = FAS_OK;
    if (!std::isfinite(h0)) st = FAS_DIVERGED;
    for (int k = 0; k < max_cycles && st == FAS_OK; ++k) {
        cycle(s, 0);
        s->n_cycles++;
        ++done;
        STCHK(norm(s, &h));
        if (res_hist) res_hist[k + 1] = h;
        if (!std::isfinite(h)) { st = FAS_DIVERGED; break; }
        if (drop_orders > 0.0 && h <= h0 * std::pow(10.0, -drop_orders)) break;
    }
    if (n_done) *n_done = done;
    HIPCHK(hipGetLastError());
    if (st == FAS_OK && drop_orders > 0.0 && !(h <= h0 * std::pow(10.0, -drop_orders)) && done == max_cycles)
        st = FAS_NOT_CONVERGED;
    if (st == FAS_DIVERGED) g_err = "residual norm is not finite";
    if (st == FAS_NOT_CONVERGED) g_err = "cycle cap reached before the requested residual drop";
    return st;
}

extern "C" fas_status fas_dual_time_step(fas_state s, double dt, double alpha_deg, int32_t max_inner,
                                         double drop_orders, double *res_hist, int32_t *n_inner) {
    if (!s || !(dt > 0.0)) return fail(FAS_EINVAL, "bad argument");
    if (s->have_un)
        for (int l = 0; l < s->nlev; ++l)
            launch_axpby_interior(s->lv[l].L, 1.0, s->lv[l].un, 0.0, nullptr, s->lv[l].unm1, 4, s->st);
    launch_axpby_interior(s->lv[0].L, 1.0, s->lv[0].u, 0.0, nullptr, s->lv[0].un, 4, s->st);
    for (int l = 1; l < s->nlev; ++l)
        launch_restrict(s->lv[l - 1].L, s->lv[l].L, s->lv[l - 1].geo, s->lv[l].geo, s->lv[l - 1].un,
                        s->lv[l].un, nullptr, s->st);
    s->bdf = s->have_un ? 2 : 1;
    s->have_un = 1;
    s->dt = dt;
    s->n_cycles = 0;
    s->p.alpha_deg = alpha_deg;
    set_phys(s);
    return fas_cycle(s, max_inner, drop_orders, res_hist, n_inner);
}

extern "C" fas_status fas_profile(fas_state s, int32_t enable) {
    if (!s) return fail(FAS_EINVAL, "null state");
    HIPCHK(hipStreamSynchronize(s->st));
    for (auto &r : s->recs) {
        s->pool.push_back(r.a);
        s->pool.push_back(r.b);
    }
    s->recs.clear();
    for (int c = 0; c < FAS_PROF_NCLASS; ++c) {
        s->prof_ms[c] = 0.0;
        s->prof_n[c] = 0;
    }
    s->prof = enable ? 1 : 0;
    return FAS_OK;
}

extern "C" fas_status fas_profile_read(fas_state s, double *ms, int64_t *count) {
    if (!s) return fail(FAS_EINVAL, "null state");
    HIPCHK(hipStreamSynchronize(s->st));
    for (auto &r : s->recs) {
        float t = 0.0f;
        HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
        s->prof_ms[r.cls] += t;
        s->prof_n[r.cls] += 1;
        s->pool.push_back(r.a);
        s->pool.push_back(r.b);
    }
    s->recs.clear();
    for (int c = 0; c < FAS_PROF_NCLASS; ++c) {
        if (ms) ms[c] = s->prof_ms[c];
        if (count) count[c] = s->prof_n[c];
    }
    return FAS_OK;
}

extern "C" const char *fas_last_error(void) { return g_err.c_str(); }
