// Host runtime behind the C ABI of include/fas.h: object lifetimes,
// parameter checks, the smoother stage loop, the FAS recursion and dual
// time stepping, all enqueued on the caller's HIP stream.
#include "fas.h"
#include "fas_internal.h"
#include "fas_dfa.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
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

namespace {

// The cycle machinery over a batch of n cases that share the cycle
// structure (model, scheme, levels, cycle type, preconditioner precision).
// A flow state is a batch of one.
struct Engine {
    int n = 0, nlev = 0;
    hipStream_t st = nullptr;
    int model = FAS_EULER, fp32 = 0, gamma = 1, nu1 = 1;
    Scheme sc;
    std::vector<BLev> lev;
    int has_src[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int bdf = 0;
    double dt = 0.0;
    int vblk = 0;               // viscous term in the preconditioner blocks (RANS)
    int freeze_mut = 0;         // fine eddy viscosity kept at its last evaluation
    int stall_window = 0;       // stall test (0: off)
    double stall_orders = 0.0, growth_limit = 0.0;
    int *d_cyc = nullptr;       // [n]
    int *d_rb = nullptr;        // [n] roll-back flags of the status update
    double *d_norm = nullptr;   // [n]
    // optional per-kernel-class timing with HIP events on the stream
    int prof = 0;
    struct Rec { int cls; hipEvent_t a, b; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    double prof_ms[FAS_PROF_NCLASS] = {0};
    int64_t prof_n[FAS_PROF_NCLASS] = {0};
};

void engine_release_events(Engine &e) {
    for (auto &r : e.recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    e.recs.clear();
    for (auto ev : e.pool) (void)hipEventDestroy(ev);
    e.pool.clear();
}

}  // namespace

// Transposed SGS solve of one level (adjoint): the level's neighbour blocks
// transposed into the slots of the cells they act on, the sweep's input and
// forward output in the sweep precision, its backward output in FP64, and
// a launch descriptor of the primal sweep over these arrays
struct TSweep {
    void *bt = nullptr, *g = nullptr, *y = nullptr;
    double *xi = nullptr;
    LevelDev host;
    BLev B;
};

struct fas_state_s {
    fas_grid g;
    fas_params p;
    int nlev;
    Phys ph;
    std::vector<LevelDev> lv;
    Engine e;
    int have_un = 0;
    double t = 0.0;             // physical time and steps taken (dual time stepping)
    int step = 0;
    Phys *d_ph = nullptr;
    LevelDev *d_lv = nullptr;             // device copy of lv
    // rigidly rotating mesh: per-level rotated geometry and the motion
    std::vector<double *> ale_geo;
    int ale = 0;
    double ale_omega = 0.0, ale_px = 0.0, ale_py = 0.0;
    std::vector<void *> allocs;
    // adjoint work arrays (padded fine level), allocated on first use
    double *a_gbar = nullptr;   // metric-plane adjoint of the node sensitivities (lazy)
    double *a_lam = nullptr, *a_g = nullptr, *a_r = nullptr, *a_z = nullptr, *a_jt = nullptr,
           *a_lam0 = nullptr, *a_dFa = nullptr, *a_dFm = nullptr, *a_dcl = nullptr,
           *a_red = nullptr, *a_out = nullptr, *a_basis = nullptr;
    double *a_smv = nullptr;    // smoother VJP: stage states and work vectors (lazy)
    double *a_mg = nullptr;     // multilevel adjoint preconditioner: 3 arrays per coarse level (lazy)
    std::vector<TSweep> a_ts;   // transposed SGS solve per level (lazy)
    double adj_tau = 0.0;       // diagonal of the physical-time term in the adjoint operator
    std::vector<double *> a_ck; // unsteady adjoint: checkpoints and the recomputation window
    // graph-replayed cycles: activity flag (read by every kernel of the
    // state), cycles done, status, initial norm, history; a private stream
    // to capture on (the state's own stream may be the legacy default)
    int *d_act = nullptr, *d_ndone = nullptr, *d_stat = nullptr;
    double *d_h0 = nullptr, *d_hist = nullptr;
    int hcap = 0;
    int *h_act = nullptr;       // pinned: two snapshots of the activity flag
    hipEvent_t ev_chunk[2] = {nullptr, nullptr};
    hipStream_t cap_st = nullptr;
};

struct fas_batch_s {
    std::vector<fas_state> states;
    Engine e;
    int own_stream = 0;
    int *d_act = nullptr, *d_ndone = nullptr, *d_stat = nullptr;
    double *d_h0 = nullptr, *d_hist = nullptr;
    int hcap = 0;
    int *h_act = nullptr;       // pinned: two snapshots of the activity flags
    hipEvent_t ev_chunk[2] = {nullptr, nullptr};
    std::vector<void *> allocs;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_cap = -1;         // max_cycles / drop the graph was captured for
    double graph_drop = 0.0;
    // concurrent case groups: sub-batches on streams of their own (empty: the
    // batch is one group), the batch's case number of each of their cases,
    // and the solve's start on the batch stream, which every group waits for
    std::vector<fas_batch> parts;
    std::vector<std::vector<int>> part_cases;
    hipEvent_t ev_start = nullptr;
    int *h_flags = nullptr;     // pinned: two activity snapshots in flight
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
    p->viscous_blocks = 0;
    p->dt_form = 1;
    p->stall_window = 0;
    p->stall_orders = 0.0;
    p->growth_limit = 1.0e8;
    p->adjoint_levels = 0;
    p->freeze_mut = 0;
}

// upload the nodes of every level (every 2^l-th node of the fine grid) and
// compute the metrics (coarse volumes agglomerated from the finer level);
// every fine volume must be positive
static fas_status grid_upload(fas_grid g, const double *x_nodes, const double *y_nodes) {
    const int W = g->ni + 1;
    for (int l = 0; l < g->nlev; ++l) {
        const int s = 1 << l;
        const Lay &L = g->lay[l];
        const int nil = L.ni, njl = L.nj;
        std::vector<double> hx((size_t)(nil + 1) * (njl + 1)), hy(hx.size());
        for (int J = 0; J <= njl; ++J)
            for (int I = 0; I <= nil; ++I) {
                hx[(size_t)J * (nil + 1) + I] = x_nodes[(size_t)(J * s) * W + I * s];
                hy[(size_t)J * (nil + 1) + I] = y_nodes[(size_t)(J * s) * W + I * s];
            }
        if (hipMemcpy(g->xn[l], hx.data(), hx.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(g->yn[l], hy.data(), hy.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemset(g->geo[l], 0, (size_t)G_NPLANES * L.NS * sizeof(double)) != hipSuccess)
            return fail(FAS_EDEVICE, "grid upload failed");
        if (l == 0) launch_geom_interior(L, g->xn[l], g->yn[l], g->geo[l], nullptr, nullptr, nullptr, 0);
        else launch_geom_interior(L, g->xn[l], g->yn[l], g->geo[l], nullptr, &g->lay[l - 1], g->geo[l - 1], 0);
        launch_geom_ghost(L, g->xn[l], g->yn[l], g->geo[l], 0);
    }
    if (hipDeviceSynchronize() != hipSuccess) return fail(FAS_EDEVICE, "geometry kernels failed");
    const Lay &L = g->lay[0];
    std::vector<double> vol(L.NS);
    if (hipMemcpy(vol.data(), g->geo[0] + (size_t)G_VOL * L.NS, L.NS * sizeof(double), hipMemcpyDeviceToHost) !=
        hipSuccess)
        return fail(FAS_EDEVICE, "volume check failed");
    for (int j = 0; j < L.nj; ++j)
        for (int i = 0; i < L.ni; ++i)
            if (!(vol[L.slot(i, j)] > 0.0))
                return fail(FAS_EINVAL, "non-positive cell volume (grid must be right-handed)");
    return FAS_OK;
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
    // the sweep addresses each per-level array with 32-bit byte offsets
    // below 2^31 (the FP64 block array is the largest: 640 bytes per slot)
    if ((size_t)BLK_NPLANES * make_lay(ni, nj, topology == FAS_CGRID ? n_wake : 0, topology).NS * 8 >=
        ((size_t)1 << 31))
        return fail(FAS_EINVAL, "grid too large (the preconditioner blocks of the fine level exceed 2 GiB)");
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
    for (int l = 0; l < n_levels; ++l) {
        int s = 1 << l;
        int nil = ni / s, njl = nj / s;
        Lay L = make_lay(nil, njl, g->nw / s, topology);
        g->lay.push_back(L);
        const size_t nn = (size_t)(nil + 1) * (njl + 1);
        double *dx = nullptr, *dy = nullptr, *geo = nullptr;
        if (hipMalloc(&dx, nn * sizeof(double)) != hipSuccess ||
            hipMalloc(&dy, nn * sizeof(double)) != hipSuccess ||
            hipMalloc(&geo, (size_t)G_NPLANES * L.NS * sizeof(double)) != hipSuccess) {
            if (dx) g->xn.push_back(dx);
            if (dy) g->yn.push_back(dy);
            if (geo) g->geo.push_back(geo);
            return cleanup(fail(FAS_ENOMEM, "grid allocation failed"));
        }
        g->xn.push_back(dx);
        g->yn.push_back(dy);
        g->geo.push_back(geo);
    }
    {
        fas_status st = grid_upload(g, x_nodes, y_nodes);
        if (st != FAS_OK) return cleanup(st);
    }
    *out = g;
    return FAS_OK;
}

extern "C" fas_status fas_grid_set_nodes(fas_grid g, const double *x_nodes, const double *y_nodes) {
    if (!g || !x_nodes || !y_nodes) return fail(FAS_EINVAL, "null argument");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != g->device) return fail(FAS_EINVAL, "grid on another device");
    return grid_upload(g, x_nodes, y_nodes);
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
    if (p->precond_fp32 != 0 && p->precond_fp32 != 1) return fail(FAS_EINVAL, "bad precond_fp32");
    if (p->viscous_blocks != 0 && p->viscous_blocks != 1) return fail(FAS_EINVAL, "bad viscous_blocks");
    if (p->dt_form != 0 && p->dt_form != 1) return fail(FAS_EINVAL, "bad dt_form");
    if (p->stall_window < 0 || !(p->stall_orders >= 0.0) || !(p->growth_limit >= 0.0))
        return fail(FAS_EINVAL, "bad stall or growth test");
    if (p->adjoint_levels < 0 || p->adjoint_levels > p->n_levels) return fail(FAS_EINVAL, "bad adjoint_levels");
    if (p->freeze_mut != 0 && p->freeze_mut != 1) return fail(FAS_EINVAL, "bad freeze_mut");
    return FAS_OK;
}

static void fill_phys(const fas_params &p, Phys &ph) {
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
    ph.cfl = p.cfl;
    ph.cfl_ramp = p.cfl_ramp;
    ph.ramp_growth = p.ramp_growth;
    ph.n_ramp = p.n_ramp;
    ph.dt_form = p.dt_form;
    ph.rans = p.model == FAS_RANS_BL;
    ph.ale = 0;
    ph.omega = ph.px = ph.py = 0.0;
}

// host parameters -> device copy; waits for the state's earlier work, which
// may still read the old values
static fas_status set_phys(fas_state s) {
    fill_phys(s->p, s->ph);
    s->ph.ale = s->ale;
    s->ph.omega = s->ale_omega;
    s->ph.px = s->ale_px;
    s->ph.py = s->ale_py;
    Engine &e = s->e;
    e.model = s->p.model;
    e.fp32 = s->p.precond_fp32;
    e.gamma = s->p.cycle_gamma;
    e.nu1 = s->p.nu1;
    e.sc = SCHEMES[s->p.scheme];
    e.vblk = s->p.viscous_blocks;
    e.freeze_mut = s->p.freeze_mut;
    e.stall_window = s->p.stall_window;
    e.stall_orders = s->p.stall_orders;
    e.growth_limit = s->p.growth_limit;
    HIPCHK(hipStreamSynchronize(e.st));
    HIPCHK(hipMemcpyAsync(s->d_ph, &s->ph, sizeof(Phys), hipMemcpyHostToDevice, e.st));
    HIPCHK(hipStreamSynchronize(e.st));
    return FAS_OK;
}

extern "C" void fas_state_destroy(fas_state s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->e.st);
    engine_release_events(s->e);
    if (s->cap_st) (void)hipStreamDestroy(s->cap_st);
    if (s->h_act) (void)hipHostFree(s->h_act);
    for (hipEvent_t ev : s->ev_chunk)
        if (ev) (void)hipEventDestroy(ev);
    for (auto p : s->allocs) (void)hipFree(p);
    delete s;
}

static BLev make_blev(const std::vector<Lay> &lays, const LevelDev *dV, const Phys *dPH, const int *act,
                      const int *cyc) {
    BLev B;
    B.k.V = dV;
    B.k.PH = dPH;
    B.k.act = act;
    B.k.cyc = cyc;
    B.k.tile0 = nullptr;
    B.k.order = nullptr;
    B.n = (int)lays.size();
    B.k.n = B.n;
    B.ntiles = 0;
    B.max_ns = B.max_ni = B.max_nj = B.max_nw = 0;
    for (const Lay &L : lays) {
        B.max_ns = std::max(B.max_ns, L.NS);
        B.max_ni = std::max(B.max_ni, L.ni);
        B.max_nj = std::max(B.max_nj, L.nj);
        B.max_nw = std::max(B.max_nw, L.nw);
    }
    B.sweep_cfg = -1;
    return B;
}

extern "C" fas_status fas_state_create(fas_grid g, const fas_params *p, const double *u0,
                                       void *stream, fas_state *out) {
    if (!g || !out || !u0) return fail(FAS_EINVAL, "null argument");
    *out = nullptr;
    STCHK(check_params(p, g->nlev));
    fas_state s = new fas_state_s();
    s->g = g;
    s->p = *p;
    s->nlev = p->n_levels;
    Engine &e = s->e;
    e.st = (hipStream_t)stream;
    e.n = 1;
    e.nlev = s->nlev;
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
        const size_t nd = (size_t)(4 * 9 + 2 + Q_NPLANES + V_NPLANES) * NS + 256;
        const size_t nb = (size_t)BLK_NPLANES * NS * 8 + (size_t)8 * NS * 8 + bnd_count(d.L) * 8;
        double *base = nullptr;
        char *bb = nullptr;
        if (hipMalloc(&base, nd * sizeof(double)) != hipSuccess) return cleanup(fail(FAS_ENOMEM, "state allocation failed"));
        s->allocs.push_back(base);
        if (hipMalloc(&bb, nb) != hipSuccess) return cleanup(fail(FAS_ENOMEM, "state allocation failed"));
        s->allocs.push_back(bb);
        if (hipMemsetAsync(base, 0, nd * sizeof(double), e.st) != hipSuccess ||
            hipMemsetAsync(bb, 0, nb, e.st) != hipSuccess)
            return cleanup(fail(FAS_EDEVICE, "state clear failed"));
        double *q = base;
        auto take = [&](size_t n) { double *r = q; q += n * NS; return r; };
        d.u = take(4); d.u0 = take(4); d.acc = take(4); d.F = take(4);
        d.src = take(4); d.ut = take(4); d.un = take(4); d.unm1 = take(4); d.ulast = take(4);
        d.dts = take(1); d.mut = take(1); d.cq = take(Q_NPLANES); d.vg = take(V_NPLANES);
        d.red = q;
        d.blk = bb;
        d.g = bb + (size_t)BLK_NPLANES * NS * 8;
        d.y = bb + (size_t)BLK_NPLANES * NS * 8 + (size_t)4 * NS * 8;
        d.bnd = bb + (size_t)BLK_NPLANES * NS * 8 + (size_t)8 * NS * 8;
        launch_fill_int(reinterpret_cast<int *>(d.bnd), (int)(2 * bnd_count(d.L)), (int)BND_SENTINEL32, e.st);
        s->lv.push_back(d);
    }
    // device descriptors: one LevelDev per level, the physics, the cycle
    // counter and the norm
    const size_t desc = (size_t)s->nlev * sizeof(LevelDev) + sizeof(Phys) + 64;
    char *dd = nullptr;
    if (hipMalloc(&dd, desc + 64) != hipSuccess) return cleanup(fail(FAS_ENOMEM, "allocation failed"));
    s->allocs.push_back(dd);
    LevelDev *dV = reinterpret_cast<LevelDev *>(dd);
    s->d_lv = dV;
    s->d_ph = reinterpret_cast<Phys *>(dd + (size_t)s->nlev * sizeof(LevelDev));
    e.d_norm = reinterpret_cast<double *>(dd + desc - 64);
    e.d_cyc = reinterpret_cast<int *>(dd + desc);
    if (hipMemcpyAsync(dV, s->lv.data(), (size_t)s->nlev * sizeof(LevelDev), hipMemcpyHostToDevice, e.st) != hipSuccess)
        return cleanup(fail(FAS_EDEVICE, "descriptor upload failed"));
    launch_fill_int(e.d_cyc, 1, 0, e.st);
    char *gc = nullptr;
    if (hipMalloc(&gc, 64) != hipSuccess) return cleanup(fail(FAS_ENOMEM, "allocation failed"));
    s->allocs.push_back(gc);
    s->d_h0 = reinterpret_cast<double *>(gc);
    s->d_act = reinterpret_cast<int *>(gc + 16);
    s->d_ndone = reinterpret_cast<int *>(gc + 20);
    s->d_stat = reinterpret_cast<int *>(gc + 24);
    e.d_rb = reinterpret_cast<int *>(gc + 28);
    launch_fill_int(s->d_act, 1, 1, e.st);
    launch_fill_int(e.d_rb, 1, 0, e.st);
    if (hipHostMalloc(reinterpret_cast<void **>(&s->h_act), 2 * sizeof(int), hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(FAS_ENOMEM, "pinned allocation failed"));
    for (hipEvent_t &ev : s->ev_chunk)
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
            return cleanup(fail(FAS_EDEVICE, "event creation failed"));
    for (int l = 0; l < s->nlev; ++l)
        e.lev.push_back(make_blev({s->lv[l].L}, dV + l, s->d_ph, s->d_act, e.d_cyc));
    if (set_phys(s) != FAS_OK) return cleanup(FAS_EDEVICE);
    launch_unpack(s->lv[0].L, u0, s->lv[0].u, 4, e.st);
    if (hipGetLastError() != hipSuccess) return cleanup(fail(FAS_EDEVICE, "kernel launch failed"));
    *out = s;
    return FAS_OK;
}

extern "C" fas_status fas_state_set_params(fas_state s, const fas_params *p) {
    if (!s) return fail(FAS_EINVAL, "null state");
    STCHK(check_params(p, s->g->nlev));
    if (p->n_levels != s->nlev) return fail(FAS_EINVAL, "n_levels cannot change after creation");
    s->p = *p;
    return set_phys(s);
}

extern "C" fas_status fas_set_motion(fas_state s, double dalpha_deg, double rate_deg, double pivot_x,
                                      double pivot_y) {
    if (!s) return fail(FAS_EINVAL, "null state");
    if (!std::isfinite(dalpha_deg) || !std::isfinite(rate_deg) || !std::isfinite(pivot_x) ||
        !std::isfinite(pivot_y))
        return fail(FAS_EINVAL, "bad motion");
    Engine &e = s->e;
    HIPCHK(hipStreamSynchronize(e.st));
    if (s->ale_geo.empty()) {
        for (int l = 0; l < s->nlev; ++l) {
            double *g = nullptr;
            HIPCHK(hipMalloc(&g, (size_t)G_NPLANES * s->lv[l].L.NS * sizeof(double)));
            s->allocs.push_back(g);
            s->ale_geo.push_back(g);
        }
    }
    const double theta = -dalpha_deg * (M_PI / 180.0);
    const double omega = -rate_deg * (M_PI / 180.0);
    const double c = std::cos(theta), sn = std::sin(theta);
    for (int l = 0; l < s->nlev; ++l) {
        launch_rotate_geometry(s->lv[l].L, s->g->geo[l], s->g->xn[l], s->g->yn[l], s->ale_geo[l], c, sn,
                               pivot_x, pivot_y, omega, e.st);
        s->lv[l].geo = s->ale_geo[l];
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(s->d_lv, s->lv.data(), (size_t)s->nlev * sizeof(LevelDev), hipMemcpyHostToDevice, e.st));
    s->ale = 1;
    s->ale_omega = omega;
    s->ale_px = pivot_x;
    s->ale_py = pivot_y;
    return set_phys(s);
}

extern "C" fas_status fas_set_state(fas_state s, const double *u, const double *un, const double *unm1, double t,
                                    double dt, int32_t step, int32_t n_cycles) {
    if (!s || !u) return fail(FAS_EINVAL, "null argument");
    if (step < 0 || n_cycles < 0) return fail(FAS_EINVAL, "negative step or cycle count");
    if (step > 0 && (!(dt > 0.0) || !std::isfinite(t) || !un || (step > 1 && !unm1)))
        return fail(FAS_EINVAL, "a time-accurate state needs dt > 0, a finite t, un and (step > 1) unm1");
    Engine &e = s->e;
    launch_unpack(s->lv[0].L, u, s->lv[0].u, 4, e.st);
    if (step > 0) {
        // the time levels of the step in progress, restricted to the coarse
        // levels exactly as fas_dual_time_step restricts them
        launch_unpack(s->lv[0].L, un, s->lv[0].un, 4, e.st);
        for (int l = 1; l < s->nlev; ++l) launch_restrict(e.lev[l - 1], e.lev[l], FLD_UN, FLD_UN, FLD_NONE, e.st);
        if (step > 1) {
            launch_unpack(s->lv[0].L, unm1, s->lv[0].unm1, 4, e.st);
            for (int l = 1; l < s->nlev; ++l)
                launch_restrict(e.lev[l - 1], e.lev[l], FLD_UNM1, FLD_UNM1, FLD_NONE, e.st);
        }
        e.bdf = step > 1 ? 2 : 1;
        e.dt = dt;
        s->have_un = 1;
        s->t = t;
    } else {
        e.bdf = 0;
        e.dt = 0.0;
        s->have_un = 0;
        s->t = 0.0;
    }
    s->step = step;
    launch_fill_int(e.d_cyc, 1, n_cycles, e.st);
    HIPCHK(hipGetLastError());
    return FAS_OK;
}

extern "C" fas_status fas_get_time_levels(fas_state s, double *un, double *unm1, double *t, double *dt,
                                          int32_t *step, int32_t *n_cycles) {
    if (!s) return fail(FAS_EINVAL, "null state");
    Engine &e = s->e;
    if (un && s->step > 0) launch_pack(s->lv[0].L, s->lv[0].un, un, 4, e.st);
    if (unm1 && s->step > 1) launch_pack(s->lv[0].L, s->lv[0].unm1, unm1, 4, e.st);
    int nc = 0;
    HIPCHK(hipMemcpyAsync(&nc, e.d_cyc, sizeof(int), hipMemcpyDeviceToHost, e.st));
    HIPCHK(hipStreamSynchronize(e.st));
    if (t) *t = s->t;
    if (dt) *dt = e.dt;
    if (step) *step = s->step;
    if (n_cycles) *n_cycles = nc;
    return FAS_OK;
}

extern "C" fas_status fas_get_state(fas_state s, double *u, double *mu_t) {
    if (!s) return fail(FAS_EINVAL, "null state");
    if (u) launch_pack(s->lv[0].L, s->lv[0].u, u, 4, s->e.st);
    if (mu_t) launch_pack(s->lv[0].L, s->lv[0].mut, mu_t, 1, s->e.st);
    HIPCHK(hipGetLastError());
    return FAS_OK;
}

extern "C" fas_status fas_get_level(fas_state s, int32_t level, double *u, double *source) {
    if (!s || level < 0 || level >= s->nlev) return fail(FAS_EINVAL, "bad level");
    const LevelDev &d = s->lv[level];
    if (u) launch_pack(d.L, d.u, u, 4, s->e.st);
    if (source) launch_pack(d.L, d.src, source, 4, s->e.st);
    HIPCHK(hipGetLastError());
    return FAS_OK;
}

extern "C" fas_status fas_handoff_pending(fas_state s, int32_t level, int64_t *n_pending) {
    if (!s || !n_pending || level < 0 || level >= s->nlev) return fail(FAS_EINVAL, "bad argument");
    const LevelDev &d = s->lv[level];
    std::vector<uint32_t> h(2 * bnd_count(d.L));
    HIPCHK(hipStreamSynchronize(s->e.st));
    HIPCHK(hipMemcpy(h.data(), d.bnd, h.size() * sizeof(uint32_t), hipMemcpyDeviceToHost));
    int64_t n = 0;
    for (uint32_t w : h) n += w != BND_SENTINEL32;
    *n_pending = n;
    return FAS_OK;
}

// ----------------------------------------------------------- building blocks
namespace {

hipEvent_t take_event(Engine &e) {
    if (!e.pool.empty()) {
        hipEvent_t ev = e.pool.back();
        e.pool.pop_back();
        return ev;
    }
    hipEvent_t ev = nullptr;
    (void)hipEventCreate(&ev);
    return ev;
}

// brackets a launch with events when profiling is on
struct Prof {
    Engine &e;
    int cls;
    hipEvent_t a = nullptr;
    Prof(Engine &e_, int c) : e(e_), cls(c) {
        if (e.prof) {
            a = take_event(e);
            (void)hipEventRecord(a, e.st);
        }
    }
    ~Prof() {
        if (a) {
            hipEvent_t b = take_event(e);
            (void)hipEventRecord(b, e.st);
            e.recs.push_back({cls, a, b});
        }
    }
};

// the Baldwin-Lomax model runs on the fine level; every RANS level carries
// the viscous flux (coarse levels with the restricted eddy viscosity)
bool fine_rans(const Engine &e, int l) { return l == 0 && e.model == FAS_RANS_BL; }
bool rans(const Engine &e) { return e.model == FAS_RANS_BL; }

double tau_of(const Engine &e) {
    if (e.bdf == 2) return 3.0 / (2.0 * e.dt);
    if (e.bdf == 1) return 1.0 / e.dt;
    return 0.0;
}

// ghosts, cell quantities, vertex gradients (fine RANS) and, on request,
// the Baldwin-Lomax eddy viscosity for the level's current solution
void prep(Engine &e, int l, bool with_bl) {
    const BLev &B = e.lev[l];
    const int rans = e.model == FAS_RANS_BL;
    launch_ghost_cq(B, rans, rans, e.st);
    if (rans) launch_vertex_gradients(B, e.st);
    if (fine_rans(e, l) && with_bl && !e.freeze_mut) {
        launch_baldwin_lomax(B, e.st);
        launch_mut_ghosts(B, e.st);
    }
}

ResArgs res_args(const Engine &e, int l, int mode, int forcing) {
    ResArgs a;
    std::memset(&a, 0, sizeof(a));
    a.fine = l == 0;
    a.viscous = rans(e);
    a.bdf = e.bdf;
    a.dt = e.dt;
    a.forcing = forcing && e.has_src[l];
    a.mode = mode;
    a.aw = e.sc.aw;
    a.fp32 = e.fp32;
    return a;
}

// F_l(u_l) (- s_l) into the level's F, eddy viscosity evaluated at u_l
void eval_F(Engine &e, int l, bool forcing) {
    prep(e, l, fine_rans(e, l));
    launch_residual(e.lev[l], res_args(e, l, 0, forcing), e.st);
}

// frozen quantities of one smoother iteration: dt*, eddy viscosity, blocks
// (prepped: the level's ghosts, cell quantities, vertex gradients and fine
// eddy viscosity already belong to its current solution)
void prepare_iteration(Engine &e, int l, bool prepped = false, bool copy_u0 = false) {
    const BLev &B = e.lev[l];
    if (!prepped) prep(e, l, fine_rans(e, l));
    Prof pr(e, FAS_PROF_BLOCKS);
    launch_blocks(B, e.sc.aw, tau_of(e), rans(e) && e.vblk, e.fp32, e.st, copy_u0 ? 1 : 0);
}

// one smoother iteration (Section 4 low-storage stages)
void smooth_once(Engine &e, int l, bool prepped = false) {
    const BLev &B = e.lev[l];
    prepare_iteration(e, l, prepped, true);      // u0 = u: the iteration's starting state
    for (int k = 0; k < e.sc.s; ++k) {
        if (k > 0) prep(e, l, false);
        ResArgs a = res_args(e, l, 1, 1);
        a.stage = k;
        a.beta = e.sc.beta[k];
        {
            Prof pr(e, FAS_PROF_RESIDUAL);
            launch_residual(B, a, e.st);
        }
        SweepArgs sw;
        sw.update = 1;
        sw.alpha = e.sc.alpha[k];
        sw.aw = e.sc.aw;
        sw.xout_acc = 0;
        Prof pr(e, FAS_PROF_SWEEP);
        launch_sgs(B, sw, e.fp32, e.st);
    }
}

// FAS cycle from level l.  prepped: a residual evaluation of level l's
// current solution (with the eddy viscosity the smoother uses) came last, so
// the first smoother iteration reuses its ghosts, cell quantities, vertex
// gradients and eddy viscosity instead of recomputing the same values
// (the coarse levels' forcing evaluation below, and the fine-level norm
// that precedes every cycle).
void cycle(Engine &e, int l, bool prepped = false) {
    const int nsm = l < e.nlev - 1 ? e.nu1 : 1;
    for (int k = 0; k < nsm; ++k) smooth_once(e, l, prepped && k == 0);
    if (l == e.nlev - 1) return;
    const BLev &f = e.lev[l], &c = e.lev[l + 1];
    eval_F(e, l, false);
    // u_{l+1} = I u_l (also kept as ut); acc_{l+1} = I r_l with the defect
    // r_l = s_l - F_l(u_l) formed per fine cell inside the restriction; on
    // RANS levels also the eddy viscosity F_l was evaluated with, frozen on
    // the coarser level until the next descent
    const RJob jobs[2] = {{FLD_U, 1.0, FLD_NONE, 0.0, FLD_U, FLD_UT},
                          {FLD_F, -1.0, e.has_src[l] ? FLD_SRC : FLD_NONE, 1.0, FLD_ACC, FLD_NONE}};
    launch_restrict_jobs(f, c, jobs, 2, rans(e) ? 1 : 0, e.st);
    if (rans(e)) launch_mut_ghosts(c, e.st);
    // s_{l+1} = F_{l+1}(u_{l+1}) + acc_{l+1}, written by the residual itself
    e.has_src[l + 1] = 0;
    prep(e, l + 1, fine_rans(e, l + 1));
    ResArgs ra = res_args(e, l + 1, 0, 0);
    ra.src_acc = 1;
    launch_residual(c, ra, e.st);
    e.has_src[l + 1] = 1;
    for (int k = 0; k < e.gamma; ++k) cycle(e, l + 1, k == 0);
    launch_prolong(f, c, e.st);
}

// fine-level residual norm of every case into e.d_norm
void eval_norm(Engine &e) {
    eval_F(e, 0, false);
    launch_norm(e.lev[0], e.d_norm, e.st);
}

fas_status norm(fas_state s, double *out) {
    eval_norm(s->e);
    HIPCHK(hipMemcpyAsync(out, s->e.d_norm, sizeof(double), hipMemcpyDeviceToHost, s->e.st));
    HIPCHK(hipStreamSynchronize(s->e.st));
    return FAS_OK;
}

fas_status profile_on(Engine &e, int enable) {
    HIPCHK(hipStreamSynchronize(e.st));
    for (auto &r : e.recs) {
        e.pool.push_back(r.a);
        e.pool.push_back(r.b);
    }
    e.recs.clear();
    for (int c = 0; c < FAS_PROF_NCLASS; ++c) {
        e.prof_ms[c] = 0.0;
        e.prof_n[c] = 0;
    }
    e.prof = enable ? 1 : 0;
    return FAS_OK;
}

fas_status profile_read(Engine &e, double *ms, int64_t *count) {
    HIPCHK(hipStreamSynchronize(e.st));
    for (auto &r : e.recs) {
        float t = 0.0f;
        HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
        e.prof_ms[r.cls] += t;
        e.prof_n[r.cls] += 1;
        e.pool.push_back(r.a);
        e.pool.push_back(r.b);
    }
    e.recs.clear();
    for (int c = 0; c < FAS_PROF_NCLASS; ++c) {
        if (ms) ms[c] = e.prof_ms[c];
        if (count) count[c] = e.prof_n[c];
    }
    return FAS_OK;
}

}  // namespace

extern "C" fas_status fas_residual(fas_state s, int32_t level, double *F_out) {
    if (!s || !F_out || level < 0 || level >= s->nlev) return fail(FAS_EINVAL, "bad argument");
    eval_F(s->e, level, true);
    launch_pack(s->lv[level].L, s->lv[level].F, F_out, 4, s->e.st);
    HIPCHK(hipGetLastError());
    return FAS_OK;
}

extern "C" fas_status fas_smooth(fas_state s, int32_t level, int32_t n_iter) {
    if (!s || level < 0 || level >= s->nlev || n_iter < 0) return fail(FAS_EINVAL, "bad argument");
    for (int k = 0; k < n_iter; ++k) smooth_once(s->e, level);
    HIPCHK(hipGetLastError());
    return FAS_OK;
}

extern "C" fas_status fas_sgs_apply(fas_state s, int32_t level, const double *r, double *x) {
    if (!s || !r || !x || level < 0 || level >= s->nlev) return fail(FAS_EINVAL, "bad argument");
    Engine &e = s->e;
    const LevelDev &d = s->lv[level];
    prepare_iteration(e, level);
    launch_unpack(d.L, r, d.F, 4, e.st);
    launch_dinv(e.lev[level], e.fp32, e.st);
    SweepArgs sw;
    std::memset(&sw, 0, sizeof(sw));
    sw.xout_acc = 1;
    launch_sgs(e.lev[level], sw, e.fp32, e.st);
    launch_pack(d.L, d.acc, x, 4, e.st);
    HIPCHK(hipGetLastError());
    return FAS_OK;
}

namespace {

// Convergence control of a solve (single state or batch): norms, history,
// activity, cycle counts and status live on the device and are updated by
// the status kernel after every cycle, so graph-replayed and directly
// launched cycles behave the same.
BatchCtl make_ctl(const Engine &e, double *h0, double *hist, int hcap, int *act, int *ndone, int *stat,
                  int max_cycles, double drop_orders) {
    BatchCtl ctl;
    ctl.nrm = e.d_norm;
    ctl.h0 = h0;
    ctl.hist = hist;
    ctl.hcap = hcap;
    ctl.act = act;
    ctl.cyc = e.d_cyc;
    ctl.ndone = ndone;
    ctl.stat = stat;
    ctl.drop_factor = drop_orders > 0.0 ? std::pow(10.0, -drop_orders) : 0.0;
    ctl.max_cycles = max_cycles;
    ctl.stall_window = e.stall_window;
    ctl.stall_factor = std::pow(10.0, -e.stall_orders);
    ctl.growth_limit = e.growth_limit;
    ctl.rb = e.d_rb;
    return ctl;
}

// one controlled cycle: keep the fine solution, cycle (right after a norm
// evaluation), norm, status update, roll-back of a case that diverged
void controlled_cycle(Engine &e, const BatchCtl &ctl) {
    launch_save_u(e.lev[0], e.st);
    cycle(e, 0, true);
    eval_norm(e);
    launch_batch_status(ctl, e.n, e.st);
    launch_rollback(e.lev[0], ctl.rb, e.st);
}

// refill every level's band hand-off array with the sentinel (after a
// diverged solve: a sweep whose bounded wait ran out may have left a
// value in a slot)
void rearm_handoff(const std::vector<LevelDev> &lv, hipStream_t st) {
    for (const LevelDev &d : lv)
        launch_fill_int(reinterpret_cast<int *>(d.bnd), (int)(2 * bnd_count(d.L)), (int)BND_SENTINEL32, st);
}

const char *status_message(int st) {
    switch (st) {
        case FAS_DIVERGED: return "residual norm is not finite or grew beyond the limit (solution rolled back)";
        case FAS_STALLED: return "residual drop stalled";
        case FAS_NOT_CONVERGED: return "cycle cap reached before the requested residual drop";
        default: return "no error";
    }
}

}  // namespace

// FAS cycles of one state under the device convergence control.  With
// use_graph the cycle, its norm and the status update are captured once per
// call (so every host-side setting in force is the one replayed) on the
// state's private stream and replayed on its own stream; the activity flag
// turns the replays after the stop into no-ops, so the iterates, history
// and count are those of the direct launches.  The host reads the flag
// every few cycles.
// Up to max_cycles replays of one cycle (launch), in chunks of four with up
// to two chunks queued: each chunk is followed by a copy of the m activity
// flags into its own pinned slot and an event, and the host waits for the
// older chunk while the newer one runs, so the device does not idle on the
// host's check.  Stops once a snapshot shows no active case (the chunk still
// queued then replays no-ops: every kernel skips inactive cases) or
// max_cycles were launched; returns with every chunk complete.
template <class Launch>
static fas_status replay_chunks(hipStream_t st, int max_cycles, const int *d_act, int m, int *h_slots,
                                hipEvent_t *ev, Launch launch) {
    constexpr int CHECK = 4;
    int launched = 0, queued = 0, head = 0;
    for (;;) {
        while (queued < 2 && launched < max_cycles) {
            const int k = std::min(CHECK, max_cycles - launched);
            for (int i = 0; i < k; ++i) STCHK(launch());
            launched += k;
            const int slot = (head + queued) & 1;
            HIPCHK(hipMemcpyAsync(h_slots + slot * m, d_act, m * sizeof(int), hipMemcpyDeviceToHost, st));
            HIPCHK(hipEventRecord(ev[slot], st));
            ++queued;
        }
        if (queued == 0) return FAS_OK;
        HIPCHK(hipEventSynchronize(ev[head]));
        int any = 0;
        for (int c = 0; c < m; ++c) any |= h_slots[head * m + c];
        head ^= 1;
        --queued;
        if (!any) {
            if (queued > 0) HIPCHK(hipEventSynchronize(ev[head]));
            return FAS_OK;
        }
    }
}

static fas_status run_cycles(fas_state s, int32_t max_cycles, double drop_orders, double *res_hist,
                             int32_t *n_done, bool use_graph) {
    Engine &e = s->e;
    if (max_cycles + 1 > s->hcap) {
        HIPCHK(hipStreamSynchronize(e.st));
        if (s->d_hist) {
            (void)hipFree(s->d_hist);
            for (auto &p : s->allocs)
                if (p == s->d_hist) p = nullptr;
        }
        s->d_hist = nullptr;
        HIPCHK(hipMalloc(&s->d_hist, (size_t)(max_cycles + 1) * sizeof(double)));
        s->allocs.push_back(s->d_hist);
        s->hcap = max_cycles + 1;
    }
    const BatchCtl ctl = make_ctl(e, s->d_h0, s->d_hist, s->hcap, s->d_act, s->d_ndone, s->d_stat, max_cycles,
                                  drop_orders);
    launch_fill_int(s->d_act, 1, 1, e.st);
    eval_norm(e);
    launch_batch_init(ctl, 1, e.st);
    HIPCHK(hipGetLastError());
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (use_graph) {
        if (!s->cap_st) HIPCHK(hipStreamCreateWithFlags(&s->cap_st, hipStreamNonBlocking));
        const hipStream_t own = e.st;
        e.st = s->cap_st;
        hipError_t er = hipStreamBeginCapture(e.st, hipStreamCaptureModeThreadLocal);
        if (er == hipSuccess) {
            controlled_cycle(e, ctl);
            er = hipStreamEndCapture(e.st, &graph);
        }
        e.st = own;
        if (er == hipSuccess) er = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (er != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail(FAS_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(er));
        }
    }
    fas_status st = replay_chunks(e.st, max_cycles, s->d_act, 1, s->h_act, s->ev_chunk, [&]() {
        if (use_graph) {
            if (hipGraphLaunch(exec, e.st) != hipSuccess) return fail(FAS_EDEVICE, "graph launch failed");
        } else {
            controlled_cycle(e, ctl);
        }
        return FAS_OK;
    });
    (void)hipStreamSynchronize(e.st);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (st != FAS_OK) return st;
    int nd = 0, stv = 0;
    HIPCHK(hipMemcpyAsync(&nd, s->d_ndone, sizeof(int), hipMemcpyDeviceToHost, e.st));
    HIPCHK(hipMemcpyAsync(&stv, s->d_stat, sizeof(int), hipMemcpyDeviceToHost, e.st));
    if (res_hist)
        HIPCHK(hipMemcpyAsync(res_hist, s->d_hist, (size_t)(max_cycles + 1) * sizeof(double), hipMemcpyDeviceToHost,
                              e.st));
    launch_fill_int(s->d_act, 1, 1, e.st);
    HIPCHK(hipStreamSynchronize(e.st));
    if (stv == FAS_DIVERGED) rearm_handoff(s->lv, e.st);
    HIPCHK(hipGetLastError());
    if (n_done) *n_done = nd;
    if (stv != FAS_OK) g_err = status_message(stv);
    return (fas_status)stv;
}

extern "C" fas_status fas_cycle(fas_state s, int32_t max_cycles, double drop_orders, double *res_hist,
                                int32_t *n_done) {
    if (!s || max_cycles < 0) return fail(FAS_EINVAL, "bad argument");
    // graph replay when there are enough cycles to repay a capture and no
    // per-launch profiling events
    return run_cycles(s, max_cycles, drop_orders, res_hist, n_done, max_cycles >= 4 && !s->e.prof);
}

extern "C" fas_status fas_dual_time_step(fas_state s, double dt, double alpha_deg, int32_t max_inner,
                                         double drop_orders, double *res_hist, int32_t *n_inner) {
    if (!s || !(dt > 0.0)) return fail(FAS_EINVAL, "bad argument");
    Engine &e = s->e;
    if (s->have_un)
        for (int l = 0; l < s->nlev; ++l) launch_axpby(e.lev[l], 1.0, FLD_UN, 0.0, FLD_NONE, FLD_UNM1, e.st);
    launch_axpby(e.lev[0], 1.0, FLD_U, 0.0, FLD_NONE, FLD_UN, e.st);
    for (int l = 1; l < s->nlev; ++l) launch_restrict(e.lev[l - 1], e.lev[l], FLD_UN, FLD_UN, FLD_NONE, e.st);
    e.bdf = s->have_un ? 2 : 1;
    s->have_un = 1;
    e.dt = dt;
    s->t += dt;
    s->step += 1;
    launch_fill_int(e.d_cyc, 1, 0, e.st);
    s->p.alpha_deg = alpha_deg;
    STCHK(set_phys(s));
    return fas_cycle(s, max_inner, drop_orders, res_hist, n_inner);
}

extern "C" fas_status fas_profile(fas_state s, int32_t enable) {
    if (!s) return fail(FAS_EINVAL, "null state");
    return profile_on(s->e, enable);
}

extern "C" fas_status fas_profile_read(fas_state s, double *ms, int64_t *count) {
    if (!s) return fail(FAS_EINVAL, "null state");
    return profile_read(s->e, ms, count);
}

// ------------------------------------------------------------------ adjoint
namespace {

fas_status ensure_adjoint(fas_state s) {
    if (s->a_lam) return FAS_OK;
    const size_t V = (size_t)4 * s->lv[0].L.NS;
    const size_t n = 9 * V + dot_scratch_size() + 16;
    double *b = nullptr;
    HIPCHK(hipMalloc(&b, n * sizeof(double)));
    s->allocs.push_back(b);
    launch_zero(b, n, s->e.st);
    double **f[9] = {&s->a_lam, &s->a_g, &s->a_r, &s->a_z, &s->a_jt, &s->a_lam0, &s->a_dFa, &s->a_dFm, &s->a_dcl};
    for (int k = 0; k < 9; ++k) *f[k] = b + k * V;
    s->a_red = b + 9 * V;
    s->a_out = s->a_red + dot_scratch_size();
    HIPCHK(hipGetLastError());
    return FAS_OK;
}

// sqrt(<a, b>) / (4 N) style scalar: <a, b> over the fine interior (host value)
fas_status fine_dot(fas_state s, const double *a, const double *b, double *out) {
    const LevelDev &d = s->lv[0];
    launch_dot(d.L, a, b, s->a_red, s->a_out + 8, s->e.st);
    HIPCHK(hipMemcpyAsync(out, s->a_out + 8, sizeof(double), hipMemcpyDeviceToHost, s->e.st));
    HIPCHK(hipStreamSynchronize(s->e.st));
    return FAS_OK;
}

// out = (dF/du + tau I)^T v at the prepared state: the steady Jacobian's
// transpose, plus the diagonal of the physical-time term of eq.
// "nonlin-eq" (s->adj_tau: 3/(2 dt) for a BDF2 step, 1/dt for the implicit
// Euler start, 0 for the steady adjoint entry points); out is overwritten
void adj_operator(fas_state s, const double *v, double *out) {
    const LevelDev &d = s->lv[0];
    launch_zero(out, (size_t)4 * d.L.NS, s->e.st);
    launch_vjp(d.L, d.geo, d.u, d.mut, s->ph, v, out, s->e.st);
    if (s->adj_tau != 0.0) launch_axpby_ptr(d.L, 1.0, out, s->adj_tau, v, out, s->e.st);
}

// a_r = a_g - (dF/du + tau I)^T a_lam at the prepared state
void adj_residual(fas_state s, const double *lam) {
    const LevelDev &d = s->lv[0];
    adj_operator(s, lam, s->a_jt);
    launch_axpby_ptr(d.L, 1.0, s->a_g, -1.0, s->a_jt, s->a_r, s->e.st);
}

// Krylov space of the adjoint GMRES (restart length)
constexpr int ADJ_KRYLOV = 200;

// Arrays of level l's transposed SGS solve (allocated on first use)
fas_status ensure_tsweep(fas_state s, int l) {
    if (s->a_ts.empty()) s->a_ts.resize(s->nlev);
    TSweep &t = s->a_ts[l];
    if (t.bt) return FAS_OK;
    const LevelDev &d = s->lv[l];
    // FP64 extents, as the level's own blocks: the sweep precision can change
    // with the parameters after the arrays exist
    const size_t NS = d.L.NS, es = sizeof(double);
    const size_t nb = (size_t)BLK_NPLANES * NS * es, nv = 4 * NS * es;
    const size_t n = nb + 2 * nv + 4 * NS * sizeof(double) + sizeof(LevelDev);
    char *p = nullptr;
    HIPCHK(hipMalloc(&p, n));
    s->allocs.push_back(p);
    HIPCHK(hipMemsetAsync(p, 0, n, s->e.st));
    t.bt = p;
    t.g = p + nb;
    t.y = p + nb + nv;
    t.xi = reinterpret_cast<double *>(p + nb + 2 * nv);
    LevelDev *dv = reinterpret_cast<LevelDev *>(p + nb + 2 * nv + 4 * NS * sizeof(double));
    t.host = d;
    t.host.blk = t.bt;
    t.host.g = t.g;
    t.host.y = t.y;
    t.host.acc = t.xi;
    HIPCHK(hipMemcpyAsync(dv, &t.host, sizeof(LevelDev), hipMemcpyHostToDevice, s->e.st));
    HIPCHK(hipStreamSynchronize(s->e.st));
    t.B = s->e.lev[l];
    t.B.k.V = dv;
    t.B.k.act = nullptr;
    t.B.k.tile0 = nullptr;
    t.B.k.order = nullptr;
    t.B.k.n = 1;
    t.B.n = 1;
    return FAS_OK;
}

// level l's transposed blocks from its current blocks; called after every
// preparation of the level's blocks that a transposed solve then uses
fas_status transpose_blocks(fas_state s, int l) {
    STCHK(ensure_tsweep(s, l));
    const LevelDev &d = s->lv[l];
    launch_blocks_t(d.L, d.blk, s->a_ts[l].bt, s->e.fp32, s->e.st);
    return FAS_OK;
}

// x = P^-T r on level l's interior (transpose_blocks first)
void sgs_transpose(fas_state s, int l, const double *r, double *x) {
    Engine &e = s->e;
    const LevelDev &d = s->lv[l];
    const TSweep &t = s->a_ts[l];
    launch_to_sweep(d.L, r, t.g, e.fp32, e.st);
    SweepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.xout_acc = 1;
    launch_sgs(t.B, a, e.fp32, e.st);
    launch_dinv_t(d.L, d.blk, t.xi, x, e.fp32, e.st);
}

// Transposed increment operator of level l: D_t P^-T (AW: increment
// P^-1 D_t r) or P^-T D_t (pARK: increment D_t P^-1 r), with the level's
// blocks and dt*; tmp is a work array of the level.
void increment_t(fas_state s, int l, const double *in, double *tmp, double *out) {
    const LevelDev &dl = s->lv[l];
    Engine &e = s->e;
    if (e.sc.aw) {
        sgs_transpose(s, l, in, tmp);
        launch_adj_update(dl.L, nullptr, 1.0, dl.dts, tmp, out, e.st);
    } else {
        launch_adj_update(dl.L, nullptr, 1.0, dl.dts, in, tmp, e.st);
        sgs_transpose(s, l, tmp, out);
    }
}

int adjoint_levels(fas_state s) { return s->p.adjoint_levels > 0 ? std::min(s->p.adjoint_levels, s->nlev) : s->nlev; }

// coarse level l's arrays of the multilevel preconditioner: restricted
// residual, correction, and the increment's work array
double *mg_array(fas_state s, int l, int k) {
    size_t off = 0;
    for (int m = 1; m < l; ++m) off += (size_t)12 * s->lv[m].L.NS;
    return s->a_mg + off + (size_t)k * 4 * s->lv[l].L.NS;
}

fas_status ensure_adjoint_mg(fas_state s, int L) {
    if (s->a_mg || L < 2) return FAS_OK;
    size_t n = 0;
    for (int m = 1; m < s->nlev; ++m) n += (size_t)12 * s->lv[m].L.NS;
    HIPCHK(hipMalloc(&s->a_mg, n * sizeof(double)));
    s->allocs.push_back(s->a_mg);
    launch_zero(s->a_mg, n, s->e.st);
    return FAS_OK;
}

// Preconditioner of the adjoint system (right preconditioning of the
// GMRES): out = M v with M = M_0^T + sum over coarse levels of
// R_0^T .. R_{l-1}^T M_l^T P_{l-1}^T .. P_0^T, the additive multilevel
// form of the FAS cycle's coarse corrections transposed (no coarse
// Jacobian is needed: each level contributes its transposed increment).
// With adjoint_levels 1 it is the fine level's transposed increment.  The
// fine part uses a_z (AW) or a_jt (pARK) as scratch; out may be a_z.
void adj_precond(fas_state s, const double *v, double *out) {
    Engine &e = s->e;
    increment_t(s, 0, v, e.sc.aw ? s->a_z : s->a_jt, out);
    const int L = adjoint_levels(s);
    if (L < 2) return;
    for (int l = 1; l < L; ++l) {                 // g_l = P^T g_{l-1}, g_0 = v
        double *g = mg_array(s, l, 0);
        launch_zero(g, (size_t)4 * s->lv[l].L.NS, e.st);
        launch_adj_prolong_t(s->lv[l - 1].L, s->lv[l].L, l == 1 ? v : mg_array(s, l - 1, 0), g, e.st);
    }
    for (int l = L - 1; l >= 1; --l) {            // w_l = M_l^T g_l + R^T w_{l+1}
        double *w = mg_array(s, l, 1);
        increment_t(s, l, mg_array(s, l, 0), mg_array(s, l, 2), w);
        if (l + 1 < L)
            launch_adj_restrict_t(s->lv[l].L, s->lv[l + 1].L, s->lv[l].geo, s->lv[l + 1].geo, mg_array(s, l + 1, 1),
                                  w, e.st);
    }
    launch_adj_restrict_t(s->lv[0].L, s->lv[1].L, s->lv[0].geo, s->lv[1].geo, mg_array(s, 1, 1), out, e.st);
}

// (dF/du)^T lam = g on the padded work arrays (a_g, a_lam) by GMRES(200)
// with restarts, right-preconditioned by the transposed smoother.  The
// exact Jacobian of the switched JST scheme is not dissipative in general
// (some eigenvalues of the preconditioned operator have negative real
// parts), so a fixed-point iteration with the smoother alone need not
// converge; GMRES only needs a nonsingular system.  hist[k] is the RMS of
// the residual estimate after k iterations.
fas_status adj_solve(fas_state s, int max_iter, double drop, double *hist, int *n_iter) {
    Engine &e = s->e;
    const LevelDev &d = s->lv[0];
    const size_t V = (size_t)4 * d.L.NS;
    const double N4 = 4.0 * d.L.ni * d.L.nj;
    constexpr int M = ADJ_KRYLOV;
    if (!s->a_basis) {
        // basis vectors, then the Gram-Schmidt scratch: coefficients and
        // reduction partials
        const size_t nb = (size_t)(M + 1) * V + (size_t)(M + 1) * (dot_scratch_size() + 2);
        HIPCHK(hipMalloc(&s->a_basis, nb * sizeof(double)));
        s->allocs.push_back(s->a_basis);
        launch_zero(s->a_basis, nb, e.st);
    }
    double *d_h = s->a_basis + (size_t)(M + 1) * V;      // M + 1 coefficients
    double *d_red = d_h + (M + 1);                         // (M + 1) * RB partials
    std::vector<double> hh(M + 1), h2(M + 1);
    auto vb = [&](int k) { return s->a_basis + (size_t)k * V; };
    // coarse levels of the preconditioner: blocks and dt* at their current
    // states (the last cycle's coarse solutions)
    const int Lmg = adjoint_levels(s);
    STCHK(ensure_adjoint_mg(s, Lmg));
    for (int l = 1; l < Lmg; ++l) prepare_iteration(e, l);
    prepare_iteration(e, 0);
    for (int l = 0; l < Lmg; ++l) STCHK(transpose_blocks(s, l));
    adj_residual(s, s->a_lam);
    double beta = 0.0;
    STCHK(fine_dot(s, s->a_r, s->a_r, &beta));
    beta = std::sqrt(beta);
    const double h0 = beta / std::sqrt(N4);
    if (hist) hist[0] = h0;
    const double target = drop > 0.0 ? beta * std::pow(10.0, -drop) : -1.0;
    int it = 0;
    double res = beta;
    std::vector<double> H((size_t)(M + 1) * M), cs(M), sn(M), gg(M + 1), y(M);
    while (it < max_iter && std::isfinite(res) && res > target && res > 0.0) {
        launch_axpby_ptr(d.L, 1.0 / res, s->a_r, 0.0, nullptr, vb(0), e.st);
        std::fill(gg.begin(), gg.end(), 0.0);
        gg[0] = res;
        int k = 0;
        for (; k < M && it < max_iter; ++k) {
            // w = (J + tau I)^T M v_k
            adj_precond(s, vb(k), s->a_r);
            adj_operator(s, s->a_r, vb(k + 1));
            // classical Gram-Schmidt, twice (all k + 1 products in one launch)
            for (int pass = 0; pass < 2; ++pass) {
                launch_mdot(d.L, vb(k + 1), vb(0), V, k + 1, d_red, d_h, e.st);
                HIPCHK(hipMemcpyAsync(pass ? h2.data() : hh.data(), d_h, (k + 1) * sizeof(double),
                                      hipMemcpyDeviceToHost, e.st));
                launch_maxpy(d.L, vb(k + 1), vb(0), V, d_h, k + 1, e.st);
            }
            HIPCHK(hipStreamSynchronize(e.st));
            for (int i = 0; i <= k; ++i) H[(size_t)i * M + k] = hh[i] + h2[i];
            double hn = 0.0;
            STCHK(fine_dot(s, vb(k + 1), vb(k + 1), &hn));
            hn = std::sqrt(hn);
            H[(size_t)(k + 1) * M + k] = hn;
            if (hn > 0.0) launch_axpby_ptr(d.L, 1.0 / hn, vb(k + 1), 0.0, nullptr, vb(k + 1), e.st);
            for (int i = 0; i < k; ++i) {
                const double a = H[(size_t)i * M + k], b = H[(size_t)(i + 1) * M + k];
                H[(size_t)i * M + k] = cs[i] * a + sn[i] * b;
                H[(size_t)(i + 1) * M + k] = -sn[i] * a + cs[i] * b;
            }
            const double a = H[(size_t)k * M + k], b = H[(size_t)(k + 1) * M + k];
            const double r = std::hypot(a, b);
            cs[k] = r > 0.0 ? a / r : 1.0;
            sn[k] = r > 0.0 ? b / r : 0.0;
            H[(size_t)k * M + k] = r;
            H[(size_t)(k + 1) * M + k] = 0.0;
            gg[k + 1] = -sn[k] * gg[k];
            gg[k] = cs[k] * gg[k];
            ++it;
            res = std::fabs(gg[k + 1]);
            if (hist) hist[it] = res / std::sqrt(N4);
            if (!(res > target) || hn == 0.0) {
                ++k;
                break;
            }
        }
        // y = H^-1 g, lam += M (V y)
        for (int i = k - 1; i >= 0; --i) {
            double t = gg[i];
            for (int j = i + 1; j < k; ++j) t -= H[(size_t)i * M + j] * y[j];
            y[i] = t / H[(size_t)i * M + i];
        }
        launch_zero(s->a_r, V, e.st);
        for (int i = 0; i < k; ++i) launch_axpby_ptr(d.L, 1.0, s->a_r, y[i], vb(i), s->a_r, e.st);
        adj_precond(s, s->a_r, s->a_z);
        launch_axpby_ptr(d.L, 1.0, s->a_lam, 1.0, s->a_z, s->a_lam, e.st);
        // true residual for the restart
        adj_residual(s, s->a_lam);
        STCHK(fine_dot(s, s->a_r, s->a_r, &res));
        res = std::sqrt(res);
        if (hist) hist[it] = res / std::sqrt(N4);
    }
    if (n_iter) *n_iter = it;
    HIPCHK(hipGetLastError());
    if (!std::isfinite(res)) return fail(FAS_DIVERGED, "adjoint residual is not finite");
    if (drop > 0.0 && res > target) return fail(FAS_NOT_CONVERGED, "adjoint iteration cap reached");
    return FAS_OK;
}

}  // namespace

extern "C" fas_status fas_forces(fas_state s, double *cl, double *cd, double *dcl_du) {
    if (!s) return fail(FAS_EINVAL, "null state");
    STCHK(ensure_adjoint(s));
    const LevelDev &d = s->lv[0];
    if (dcl_du) launch_zero(s->a_dcl, (size_t)4 * d.L.NS, s->e.st);
    launch_forces(d.L, d.geo, d.u, s->ph, s->a_out, dcl_du ? s->a_dcl : nullptr, s->e.st);
    double h[6];
    HIPCHK(hipMemcpyAsync(h, s->a_out, sizeof(h), hipMemcpyDeviceToHost, s->e.st));
    if (dcl_du) launch_pack(d.L, s->a_dcl, dcl_du, 4, s->e.st);
    HIPCHK(hipStreamSynchronize(s->e.st));
    if (cl) *cl = h[0];
    if (cd) *cd = h[1];
    return FAS_OK;
}

extern "C" fas_status fas_vjp(fas_state s, const double *lam, double *out) {
    if (!s || !lam || !out) return fail(FAS_EINVAL, "null argument");
    if (s->ale) return fail(FAS_EINVAL, "the adjoint is for fixed meshes");
    STCHK(ensure_adjoint(s));
    const LevelDev &d = s->lv[0];
    prep(s->e, 0, fine_rans(s->e, 0));
    launch_unpack(d.L, lam, s->a_lam, 4, s->e.st);
    launch_zero(s->a_jt, (size_t)4 * d.L.NS, s->e.st);
    launch_vjp(d.L, d.geo, d.u, d.mut, s->ph, s->a_lam, s->a_jt, s->e.st);
    launch_pack(d.L, s->a_jt, out, 4, s->e.st);
    HIPCHK(hipGetLastError());
    return FAS_OK;
}

// Transpose of one fine-level smoother iteration at frozen dt*, blocks and
// eddy viscosity (the quantities the iteration fixes at its start).  With
// u_0 = u, acc_0 = f^v(u_0) and, per stage i = 1..s,
//     u_i = u_0 - alpha_i x_i,  x_i = W^-1 (dt* r_{i-1}) (AW) or dt* P^-1 r_{i-1}
//     r_{i-1} = f^c(u_{i-1}) + acc_{i-1},
//     acc_i = beta_{i+1} f^v(u_i) + (1 - beta_{i+1}) acc_{i-1}   (i < s),
// the reverse sweep carries w = adjoint of u_i and a = adjoint of acc_i:
//     i = s .. 1:  (i < s) w += beta_{i+1} J_v(u_i)^T a, a *= 1 - beta_{i+1}
//                  out += w;  xbar = -alpha_i w
//                  rbar = dt* P^-T xbar (AW) or P^-T (dt* xbar)
//                  w = J_c(u_{i-1})^T rbar;  a += rbar
//     out += w + J_v(u_0)^T a.
extern "C" fas_status fas_vjp_smooth(fas_state s, const double *lam, double *out) {
    if (!s || !lam || !out) return fail(FAS_EINVAL, "null argument");
    if (s->ale) return fail(FAS_EINVAL, "the adjoint is for fixed meshes");
    if (s->e.bdf != 0) return fail(FAS_EINVAL, "the smoother adjoint is for steady states");
    STCHK(ensure_adjoint(s));
    Engine &e = s->e;
    const LevelDev &d = s->lv[0];
    const size_t V = (size_t)4 * d.L.NS;
    const int ns = e.sc.s;
    if (!s->a_smv) {
        HIPCHK(hipMalloc(&s->a_smv, (size_t)(5 + 6) * V * sizeof(double)));
        s->allocs.push_back(s->a_smv);
        launch_zero(s->a_smv, (size_t)(5 + 6) * V, e.st);
    }
    double *stage[5];
    for (int k = 0; k < 5; ++k) stage[k] = s->a_smv + (size_t)k * V;
    double *w = s->a_smv + 5 * V, *ab = w + V, *rb = ab + V, *xb = rb + V, *tmp = xb + V, *acc = tmp + V;
    // forward iteration from the current solution, keeping u_0 .. u_{s-1}
    const BLev &B = e.lev[0];
    prepare_iteration(e, 0, false, true);
    launch_axpby_ptr(d.L, 1.0, d.u, 0.0, nullptr, stage[0], e.st);
    for (int k = 0; k < ns; ++k) {
        if (k > 0) prep(e, 0, false);
        ResArgs a = res_args(e, 0, 1, 1);
        a.stage = k;
        a.beta = e.sc.beta[k];
        launch_residual(B, a, e.st);
        SweepArgs sw;
        std::memset(&sw, 0, sizeof(sw));
        sw.update = 1;
        sw.alpha = e.sc.alpha[k];
        sw.aw = e.sc.aw;
        launch_sgs(B, sw, e.fp32, e.st);
        if (k + 1 < ns) launch_axpby_ptr(d.L, 1.0, d.u, 0.0, nullptr, stage[k + 1], e.st);
    }
    // the state keeps its solution
    launch_axpby(B, 1.0, FLD_U0, 0.0, FLD_NONE, FLD_U, e.st);
    STCHK(transpose_blocks(s, 0));
    // reverse sweep
    launch_unpack(d.L, lam, w, 4, e.st);
    launch_zero(ab, V, e.st);
    launch_zero(acc, V, e.st);
    for (int i = ns; i >= 1; --i) {
        if (i < ns) {
            const double b = e.sc.beta[i];      // beta_{i+1} in the paper's 1-based stage count
            launch_zero(tmp, V, e.st);
            launch_vjp(d.L, d.geo, stage[i], d.mut, s->ph, ab, tmp, e.st, 2);
            launch_axpby_ptr(d.L, 1.0, w, b, tmp, w, e.st);
            launch_axpby_ptr(d.L, 1.0 - b, ab, 0.0, nullptr, ab, e.st);
        }
        launch_axpby_ptr(d.L, 1.0, acc, 1.0, w, acc, e.st);
        launch_axpby_ptr(d.L, -e.sc.alpha[i - 1], w, 0.0, nullptr, xb, e.st);
        increment_t(s, 0, xb, s->a_z, rb);
        launch_zero(w, V, e.st);
        launch_vjp(d.L, d.geo, stage[i - 1], d.mut, s->ph, rb, w, e.st, 1);
        launch_axpby_ptr(d.L, 1.0, ab, 1.0, rb, ab, e.st);
    }
    launch_zero(tmp, V, e.st);
    launch_vjp(d.L, d.geo, stage[0], d.mut, s->ph, ab, tmp, e.st, 2);
    launch_axpby_ptr(d.L, 1.0, acc, 1.0, w, acc, e.st);
    launch_axpby_ptr(d.L, 1.0, acc, 1.0, tmp, acc, e.st);
    launch_pack(d.L, acc, out, 4, e.st);
    HIPCHK(hipGetLastError());
    return FAS_OK;
}

// dx, dy = (dG/dX)^T ((dF/dG)^T lam (+ dC_L/dG)) at the prepared fine level
static fas_status node_gradient(fas_state s, const double *lam, bool with_lift, double *dx, double *dy) {
    const LevelDev &d = s->lv[0];
    const size_t ng = (size_t)(G_YC + 1) * d.L.NS;
    if (!s->a_gbar) {
        HIPCHK(hipMalloc(&s->a_gbar, ng * sizeof(double)));
        s->allocs.push_back(s->a_gbar);
    }
    const size_t nn = (size_t)(d.L.ni + 1) * (d.L.nj + 1);
    launch_zero(s->a_gbar, ng, s->e.st);
    launch_vjp_geo(d.L, d.geo, d.u, d.mut, s->ph, lam, s->a_gbar, s->e.st);
    if (with_lift) launch_forces_geo(d.L, d.geo, d.u, s->ph, s->a_gbar, s->e.st);
    launch_zero(dx, nn, s->e.st);
    launch_zero(dy, nn, s->e.st);
    launch_geo_nodes(d.L, s->g->xn[0], s->g->yn[0], s->a_gbar, dx, dy, s->e.st);
    HIPCHK(hipGetLastError());
    return FAS_OK;
}

extern "C" fas_status fas_vjp_nodes(fas_state s, const double *lam, double *dx, double *dy) {
    if (!s || !lam || !dx || !dy) return fail(FAS_EINVAL, "null argument");
    if (s->ale) return fail(FAS_EINVAL, "the adjoint is for fixed meshes");
    STCHK(ensure_adjoint(s));
    const LevelDev &d = s->lv[0];
    prep(s->e, 0, fine_rans(s->e, 0));
    launch_unpack(d.L, lam, s->a_jt, 4, s->e.st);
    return node_gradient(s, s->a_jt, false, dx, dy);
}

extern "C" fas_status fas_param_partials(fas_state s, double *dF_dalpha, double *dF_dmach, double *dcl_dparam) {
    if (!s) return fail(FAS_EINVAL, "null state");
    if (s->ale) return fail(FAS_EINVAL, "the adjoint is for fixed meshes");
    STCHK(ensure_adjoint(s));
    const LevelDev &d = s->lv[0];
    prep(s->e, 0, fine_rans(s->e, 0));
    launch_param_partials(d.L, d.geo, d.u, d.mut, s->ph, s->p.reynolds, s->a_dFa, s->a_dFm, s->e.st);
    if (dF_dalpha) launch_pack(d.L, s->a_dFa, dF_dalpha, 4, s->e.st);
    if (dF_dmach) launch_pack(d.L, s->a_dFm, dF_dmach, 4, s->e.st);
    if (dcl_dparam) {
        launch_forces(d.L, d.geo, d.u, s->ph, s->a_out, nullptr, s->e.st);
        double h[6];
        HIPCHK(hipMemcpyAsync(h, s->a_out, sizeof(h), hipMemcpyDeviceToHost, s->e.st));
        HIPCHK(hipStreamSynchronize(s->e.st));
        dcl_dparam[0] = h[2];
        dcl_dparam[1] = h[3];
    }
    HIPCHK(hipGetLastError());
    return FAS_OK;
}

extern "C" fas_status fas_sgs_apply_transpose(fas_state s, const double *r, double *x) {
    if (!s || !r || !x) return fail(FAS_EINVAL, "null argument");
    STCHK(ensure_adjoint(s));
    const LevelDev &d = s->lv[0];
    prepare_iteration(s->e, 0);
    STCHK(transpose_blocks(s, 0));
    launch_unpack(d.L, r, s->a_r, 4, s->e.st);
    sgs_transpose(s, 0, s->a_r, s->a_z);
    launch_pack(d.L, s->a_z, x, 4, s->e.st);
    HIPCHK(hipGetLastError());
    return FAS_OK;
}

extern "C" fas_status fas_adjoint_solve(fas_state s, const double *rhs, double *lam, int32_t max_iter,
                                        double drop_orders, double *res_hist, int32_t *n_iter) {
    if (!s || !rhs || !lam || max_iter < 0) return fail(FAS_EINVAL, "bad argument");
    if (s->ale) return fail(FAS_EINVAL, "the adjoint is for fixed meshes");
    STCHK(ensure_adjoint(s));
    const LevelDev &d = s->lv[0];
    launch_unpack(d.L, rhs, s->a_g, 4, s->e.st);
    launch_unpack(d.L, lam, s->a_lam, 4, s->e.st);
    int n = 0;
    fas_status st = adj_solve(s, max_iter, drop_orders, res_hist, &n);
    if (n_iter) *n_iter = n;
    launch_pack(d.L, s->a_lam, lam, 4, s->e.st);
    HIPCHK(hipStreamSynchronize(s->e.st));
    return st;
}

extern "C" fas_status fas_lift_gradient(fas_state s, int32_t max_iter, double drop_orders, double *cl,
                                        double *grad, double *res_hist, int32_t *n_iter) {
    if (!s || !grad || max_iter < 0) return fail(FAS_EINVAL, "bad argument");
    if (s->ale) return fail(FAS_EINVAL, "the adjoint is for fixed meshes");
    STCHK(ensure_adjoint(s));
    Engine &e = s->e;
    const LevelDev &d = s->lv[0];
    const size_t V = (size_t)4 * d.L.NS;
    // dC_L/du and the explicit partials at the current state
    launch_zero(s->a_dcl, V, e.st);
    launch_forces(d.L, d.geo, d.u, s->ph, s->a_out, s->a_dcl, e.st);
    double h[6];
    HIPCHK(hipMemcpyAsync(h, s->a_out, sizeof(h), hipMemcpyDeviceToHost, e.st));
    HIPCHK(hipStreamSynchronize(e.st));
    // (dF/du)^T lam = -dC_L/du
    launch_axpby_ptr(d.L, -1.0, s->a_dcl, 0.0, nullptr, s->a_g, e.st);
    launch_zero(s->a_lam, V, e.st);
    int n = 0;
    fas_status st = adj_solve(s, max_iter, drop_orders, res_hist, &n);
    if (n_iter) *n_iter = n;
    if (st != FAS_OK && st != FAS_NOT_CONVERGED) return st;
    launch_param_partials(d.L, d.geo, d.u, d.mut, s->ph, s->p.reynolds, s->a_dFa, s->a_dFm, e.st);
    double la = 0.0, lm = 0.0;
    STCHK(fine_dot(s, s->a_lam, s->a_dFa, &la));
    STCHK(fine_dot(s, s->a_lam, s->a_dFm, &lm));
    if (cl) *cl = h[0];
    grad[0] = h[2] + la;
    grad[1] = h[3] + lm;
    return st;
}

extern "C" fas_status fas_lift_gradient_nodes(fas_state s, int32_t max_iter, double drop_orders, double *cl,
                                              double *grad, double *dcl_dx, double *dcl_dy, double *res_hist,
                                              int32_t *n_iter) {
    if (!s || !grad || !dcl_dx || !dcl_dy || max_iter < 0) return fail(FAS_EINVAL, "bad argument");
    const fas_status st = fas_lift_gradient(s, max_iter, drop_orders, cl, grad, res_hist, n_iter);
    if (st != FAS_OK && st != FAS_NOT_CONVERGED) return st;
    prep(s->e, 0, fine_rans(s->e, 0));
    STCHK(node_gradient(s, s->a_lam, true, dcl_dx, dcl_dy));
    HIPCHK(hipStreamSynchronize(s->e.st));
    return st;
}

// Discrete adjoint of dual time stepping (eq. "nonlin-eq": implicit Euler on
// the first step, BDF2 after it) on a fixed mesh, for the time-averaged lift
// J = (1/N) sum_{n=1..N} C_L(u^n, alpha_n) of N steps started from the
// state's steady solution u^0 at alpha_0.  Step n solves
//     R^n = F(u^n; alpha_n, M) + T^n = 0,
//     T^1 = (u^1 - u^0) / dt,  T^n = (3 u^n - 4 u^{n-1} + u^{n-2}) / (2 dt),
// and u^0 solves F(u^0; alpha_0, M) = 0.  Backwards from n = N to 0:
//     (dF/du|_n + tau_n I)^T lam^n = -(1/N) dC_L/du|_n (n >= 1)
//         - (dT^{n+1}/du^n) lam^{n+1} - (dT^{n+2}/du^n) lam^{n+2}
// with tau_1 = 1/dt, tau_n = 3/(2 dt), tau_0 = 0, dT^{n+1}/du^n = -2/dt
// (-1/dt for n = 0) and dT^{n+2}/du^n = 1/(2 dt); then
//     dJ/dM = sum_n [(1/N) dC_L/dM|_n + lam^n . dF/dM|_n],
//     dJ/dalpha_n = (1/N) dC_L/dalpha|_n + lam^n . dF/dalpha|_n.
// States are kept at every checkpoint_every-th step (each checkpoint holds
// u^k and u^{k-1}); the reverse pass recomputes the states between two
// checkpoints from the earlier one (the same dual time steps, so bitwise the
// same states) into a window and runs the adjoint steps of that segment.
extern "C" fas_status fas_unsteady_lift_gradient(fas_state s, int32_t n_steps, double dt, const double *alpha_deg,
                                                 int32_t max_inner, double inner_drop, int32_t checkpoint_every,
                                                 int32_t adj_max_iter, double adj_drop, double *J, double *dJ_dmach,
                                                 double *dJ_dalpha, int32_t *adj_iters, double *adj_orders,
                                                 int32_t *recomputed_steps) {
    if (!s || !alpha_deg || !J || !dJ_dmach || !dJ_dalpha || n_steps < 1 || !(dt > 0.0) || max_inner < 1 ||
        checkpoint_every < 1 || adj_max_iter < 0)
        return fail(FAS_EINVAL, "bad argument");
    if (s->ale) return fail(FAS_EINVAL, "the adjoint is for fixed meshes");
    if (s->e.bdf != 0 || s->step != 0) return fail(FAS_EINVAL, "the unsteady adjoint starts from a steady state");
    for (int n = 0; n <= n_steps; ++n)
        if (!std::isfinite(alpha_deg[n])) return fail(FAS_EINVAL, "bad angle");
    STCHK(ensure_adjoint(s));
    Engine &e = s->e;
    const LevelDev &d = s->lv[0];
    const size_t V = (size_t)4 * d.L.NS;
    const int N = n_steps, K = checkpoint_every;
    const int nck = N / K + 1;                 // checkpoints at steps 0, K, 2K, ... <= N
    // buffers: per checkpoint u^k and u^{k-1}; a window of K states; the
    // adjoints lam^{n+1} and lam^{n+2}; the final state and its time levels
    const size_t need = (size_t)2 * nck + K + 2 + 3;
    for (double *p : s->a_ck) (void)hipFree(p);
    s->a_ck.clear();
    for (size_t k = 0; k < need; ++k) {
        double *p = nullptr;
        if (hipMalloc(&p, V * sizeof(double)) != hipSuccess) {
            for (double *q : s->a_ck) (void)hipFree(q);
            s->a_ck.clear();
            return fail(FAS_ENOMEM, "unsteady adjoint storage");
        }
        s->a_ck.push_back(p);
        launch_zero(p, V, e.st);
    }
    double **ck = s->a_ck.data();                          // [2 nck]: u^k, u^{k-1}
    double **win = ck + 2 * nck;                           // [K]
    double *l1 = win[K], *l2 = win[K + 1];                 // lam^{n+1}, lam^{n+2}
    double *fin_u = win[K + 2], *fin_un = win[K + 3], *fin_unm1 = win[K + 4];
    const fas_params p0 = s->p;
    auto set_alpha = [&](double a) {
        s->p.alpha_deg = a;
        return set_phys(s);
    };
    auto copy = [&](const double *src, double *dst) { launch_axpby_ptr(d.L, 1.0, src, 0.0, nullptr, dst, e.st); };
    // ------------------------------------------------------------ forward
    const double w = 1.0 / N;
    double Jsum = 0.0;
    copy(d.u, ck[0]);
    STCHK(set_alpha(alpha_deg[0]));
    for (int n = 1; n <= N; ++n) {
        int nd = 0;
        const fas_status st = fas_dual_time_step(s, dt, alpha_deg[n], max_inner, inner_drop, nullptr, &nd);
        if (st == FAS_DIVERGED || st == FAS_EDEVICE || st == FAS_EINVAL || st == FAS_ENOMEM) return st;
        launch_forces(d.L, d.geo, d.u, s->ph, s->a_out, nullptr, e.st);
        double h[6];
        HIPCHK(hipMemcpyAsync(h, s->a_out, sizeof(h), hipMemcpyDeviceToHost, e.st));
        HIPCHK(hipStreamSynchronize(e.st));
        Jsum += w * h[0];
        if (n % K == 0) {
            copy(d.u, ck[2 * (n / K)]);
            copy(d.un, ck[2 * (n / K) + 1]);
        }
    }
    copy(d.u, fin_u);
    copy(d.un, fin_un);
    if (N >= 2) copy(d.unm1, fin_unm1);
    const double fin_t = s->t;
    int fin_cyc = 0;
    HIPCHK(hipMemcpyAsync(&fin_cyc, e.d_cyc, sizeof(int), hipMemcpyDeviceToHost, e.st));
    HIPCHK(hipStreamSynchronize(e.st));
    std::vector<double> hist((size_t)adj_max_iter + 1);
    // ------------------------------------------------------------ reverse
    launch_zero(l1, V, e.st);
    launch_zero(l2, V, e.st);
    double dM = 0.0;
    for (int n = 0; n <= N; ++n) dJ_dalpha[n] = 0.0;
    int recomputed = 0;
    for (int seg = N / K; seg >= 0; --seg) {
        const int k0 = seg * K, k1 = std::min(k0 + K, N + 1);
        // the segment's states u^{k0} .. u^{k1 - 1} into the window
        if (k0 == 0) {
            copy(ck[0], d.u);
            e.bdf = 0;
            e.dt = 0.0;
            s->have_un = 0;
            s->t = 0.0;
            s->step = 0;
        } else {
            copy(ck[2 * seg], d.u);
            copy(ck[2 * seg + 1], d.un);
            for (int l = 1; l < s->nlev; ++l) launch_restrict(e.lev[l - 1], e.lev[l], FLD_UN, FLD_UN, FLD_NONE, e.st);
            e.bdf = k0 > 1 ? 2 : 1;
            e.dt = dt;
            s->have_un = 1;
            s->t = k0 * dt;
            s->step = k0;
        }
        STCHK(set_alpha(alpha_deg[k0]));
        copy(d.u, win[0]);
        for (int n = k0 + 1; n < k1; ++n) {
            int nd = 0;
            const fas_status st = fas_dual_time_step(s, dt, alpha_deg[n], max_inner, inner_drop, nullptr, &nd);
            if (st == FAS_DIVERGED || st == FAS_EDEVICE || st == FAS_EINVAL || st == FAS_ENOMEM) return st;
            copy(d.u, win[n - k0]);
            ++recomputed;
        }
        for (int n = k1 - 1; n >= k0; --n) {
            copy(win[n - k0], d.u);
            e.bdf = n >= 2 ? 2 : n;
            e.dt = n >= 1 ? dt : 0.0;
            s->adj_tau = n >= 2 ? 1.5 / dt : n == 1 ? 1.0 / dt : 0.0;
            STCHK(set_alpha(alpha_deg[n]));
            prep(e, 0, fine_rans(e, 0));          // eddy viscosity frozen at u^n
            // right-hand side: -(1/N) dC_L/du + c1 lam^{n+1} - (1/(2 dt)) lam^{n+2}
            launch_zero(s->a_dcl, V, e.st);
            launch_forces(d.L, d.geo, d.u, s->ph, s->a_out, s->a_dcl, e.st);
            double h[6];
            HIPCHK(hipMemcpyAsync(h, s->a_out, sizeof(h), hipMemcpyDeviceToHost, e.st));
            HIPCHK(hipStreamSynchronize(e.st));
            const double c1 = n >= 1 ? 2.0 / dt : 1.0 / dt;
            launch_axpby_ptr(d.L, n >= 1 ? -w : 0.0, s->a_dcl, c1, l1, s->a_g, e.st);
            launch_axpby_ptr(d.L, 1.0, s->a_g, -0.5 / dt, l2, s->a_g, e.st);
            copy(l1, s->a_lam);                   // initial guess: the later step's adjoint
            // the preconditioner's dt* at the full c*, whatever cycle count
            // the (re)computed step left behind
            launch_fill_int(e.d_cyc, 1, 1 << 24, e.st);
            int it = 0;
            const fas_status st = adj_solve(s, adj_max_iter, adj_drop, hist.data(), &it);
            if (adj_iters) adj_iters[n] = it;
            if (adj_orders) {
                double lo = hist[0];
                for (int q = 0; q <= it; ++q) lo = std::min(lo, hist[q]);
                adj_orders[n] = hist[0] > 0.0 && lo > 0.0 ? std::log10(hist[0] / lo) : 0.0;
            }
            if (st != FAS_OK && st != FAS_NOT_CONVERGED) {
                s->adj_tau = 0.0;
                s->p = p0;
                (void)set_phys(s);
                return st;
            }
            launch_param_partials(d.L, d.geo, d.u, d.mut, s->ph, s->p.reynolds, s->a_dFa, s->a_dFm, e.st);
            double la = 0.0, lm = 0.0;
            STCHK(fine_dot(s, s->a_lam, s->a_dFa, &la));
            STCHK(fine_dot(s, s->a_lam, s->a_dFm, &lm));
            dJ_dalpha[n] = la + (n >= 1 ? w * h[2] : 0.0);
            dM += lm + (n >= 1 ? w * h[3] : 0.0);
            copy(l1, l2);
            copy(s->a_lam, l1);
        }
    }
    s->adj_tau = 0.0;
    // the state as the forward pass left it: u^N, its time levels and clock
    copy(fin_u, d.u);
    copy(fin_un, d.un);
    for (int l = 1; l < s->nlev; ++l) launch_restrict(e.lev[l - 1], e.lev[l], FLD_UN, FLD_UN, FLD_NONE, e.st);
    if (N >= 2) {
        copy(fin_unm1, d.unm1);
        for (int l = 1; l < s->nlev; ++l) launch_restrict(e.lev[l - 1], e.lev[l], FLD_UNM1, FLD_UNM1, FLD_NONE, e.st);
    }
    e.bdf = N >= 2 ? 2 : 1;
    e.dt = dt;
    s->have_un = 1;
    s->t = fin_t;
    s->step = N;
    launch_fill_int(e.d_cyc, 1, fin_cyc, e.st);
    STCHK(set_alpha(alpha_deg[N]));
    for (double *q : s->a_ck) (void)hipFree(q);
    s->a_ck.clear();
    HIPCHK(hipStreamSynchronize(e.st));
    *J = Jsum;
    *dJ_dmach = dM;
    if (recomputed_steps) *recomputed_steps = recomputed;
    return FAS_OK;
}

// -------------------------------------------------------------------- batch
extern "C" void fas_batch_destroy(fas_batch b) {
    if (!b) return;
    for (fas_batch p : b->parts) fas_batch_destroy(p);
    if (b->ev_start) (void)hipEventDestroy(b->ev_start);
    if (b->h_flags) (void)hipHostFree(b->h_flags);
    if (b->e.st) (void)hipStreamSynchronize(b->e.st);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    engine_release_events(b->e);
    for (auto p : b->allocs) (void)hipFree(p);
    if (b->h_act) (void)hipHostFree(b->h_act);
    for (hipEvent_t ev : b->ev_chunk)
        if (ev) (void)hipEventDestroy(ev);
    if (b->own_stream && b->e.st) (void)hipStreamDestroy(b->e.st);
    delete b;
}

static void drop_graph(fas_batch b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_cap = -1;
}

// time n sweeps of one level in configuration cfg (update off: only the
// sweep's own scratch vector y is written)
static fas_status time_sweep(Engine &e, int l, int cfg, int reps, float *ms) {
    BLev B = e.lev[l];
    B.sweep_cfg = cfg;
    SweepArgs sw;
    std::memset(&sw, 0, sizeof(sw));
    hipEvent_t a = nullptr, c = nullptr;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&c));
    launch_sgs(B, sw, e.fp32, e.st);     // warm-up
    (void)hipEventRecord(a, e.st);
    for (int k = 0; k < reps; ++k) launch_sgs(B, sw, e.fp32, e.st);
    (void)hipEventRecord(c, e.st);
    hipError_t er = hipEventSynchronize(c);
    if (er == hipSuccess) er = hipEventElapsedTime(ms, a, c);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(c);
    if (er != hipSuccess) return fail(FAS_EDEVICE, std::string("sweep timing failed: ") + hipGetErrorString(er));
    return FAS_OK;
}

extern "C" fas_status fas_batch_create(int32_t n, const fas_state *states, void *stream, int32_t autotune,
                                       int32_t groups, fas_batch *out) {
    if (!out || !states || n < 1) return fail(FAS_EINVAL, "bad argument");
    *out = nullptr;
    const fas_state s0 = states[0];
    if (!s0) return fail(FAS_EINVAL, "null state");
    for (int c = 0; c < n; ++c) {
        const fas_state s = states[c];
        if (!s) return fail(FAS_EINVAL, "null state");
        if (s->g->device != s0->g->device) return fail(FAS_EINVAL, "states on different devices");
        if (s->p.model != s0->p.model || s->p.scheme != s0->p.scheme || s->nlev != s0->nlev ||
            s->p.cycle_gamma != s0->p.cycle_gamma || s->p.nu1 != s0->p.nu1 ||
            s->p.precond_fp32 != s0->p.precond_fp32 || s->p.viscous_blocks != s0->p.viscous_blocks ||
            s->p.freeze_mut != s0->p.freeze_mut ||
            s->p.stall_window != s0->p.stall_window || s->p.stall_orders != s0->p.stall_orders ||
            s->p.growth_limit != s0->p.growth_limit)
            return fail(FAS_EINVAL, "batched states must share model, scheme, levels, cycle, precision, "
                                    "preconditioner form, turbulence freezing and stopping tests");
        if (s->e.bdf != 0 || s->ale)
            return fail(FAS_EINVAL, "batched states must be steady on fixed meshes (no dual time step, no motion)");
        for (int k = 0; k < c; ++k)
            if (states[k] == s) return fail(FAS_EINVAL, "a state appears twice in the batch");
    }
    if (groups < 0) return fail(FAS_EINVAL, "bad group count");
    for (int c = 0; c < n; ++c) HIPCHK(hipStreamSynchronize(states[c]->e.st));
    fas_batch b = new fas_batch_s();
    b->states.assign(states, states + n);
    Engine &e = b->e;
    auto cleanup = [&](fas_status st) {
        fas_batch_destroy(b);
        return st;
    };
    if (stream) {
        e.st = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&e.st, hipStreamNonBlocking) != hipSuccess)
            return cleanup(fail(FAS_EDEVICE, "stream creation failed"));
        b->own_stream = 1;
    }
    if (groups > 1 && n > 1) {
        // cases by descending hyperplane-chain length (ni + nj), dealt to the
        // groups in turn, so every group holds long and short chains
        const int G = std::min<int>(groups, n);
        std::vector<int> ord(n);
        for (int c = 0; c < n; ++c) ord[c] = c;
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b2) {
            const Lay &La = states[a]->lv[0].L, &Lb = states[b2]->lv[0].L;
            return La.ni + La.nj > Lb.ni + Lb.nj;
        });
        b->part_cases.assign(G, {});
        for (int k = 0; k < n; ++k) b->part_cases[k % G].push_back(ord[k]);
        for (int g = 0; g < G; ++g) {
            std::vector<fas_state> sub;
            for (int c : b->part_cases[g]) sub.push_back(states[c]);
            fas_batch p = nullptr;
            const fas_status st = fas_batch_create((int32_t)sub.size(), sub.data(), nullptr, autotune, 1, &p);
            if (st != FAS_OK) return cleanup(st);
            b->parts.push_back(p);
        }
        e.n = n;
        e.nlev = s0->nlev;
        if (hipEventCreateWithFlags(&b->ev_start, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&b->h_flags), (size_t)2 * n * sizeof(int),
                          hipHostMallocDefault) != hipSuccess)
            return cleanup(fail(FAS_EDEVICE, "batch set-up failed"));
        *out = b;
        return FAS_OK;
    }
    e.n = n;
    e.nlev = s0->nlev;
    e.model = s0->p.model;
    e.fp32 = s0->p.precond_fp32;
    e.gamma = s0->p.cycle_gamma;
    e.nu1 = s0->p.nu1;
    e.sc = SCHEMES[s0->p.scheme];
    e.vblk = s0->p.viscous_blocks;
    e.freeze_mut = s0->p.freeze_mut;
    e.stall_window = s0->p.stall_window;
    e.stall_orders = s0->p.stall_orders;
    e.growth_limit = s0->p.growth_limit;
    // device arrays: per level n descriptors, n physics records, control
    const size_t nl = (size_t)e.nlev * n;
    const size_t bytes = nl * sizeof(LevelDev) + (size_t)n * sizeof(Phys) + (size_t)n * (5 * sizeof(int) + 2 * sizeof(double)) + 256;
    char *dd = nullptr;
    if (hipMalloc(&dd, bytes) != hipSuccess) return cleanup(fail(FAS_ENOMEM, "batch allocation failed"));
    b->allocs.push_back(dd);
    LevelDev *dV = reinterpret_cast<LevelDev *>(dd);
    Phys *dPH = reinterpret_cast<Phys *>(dd + nl * sizeof(LevelDev));
    char *q = dd + nl * sizeof(LevelDev) + (size_t)n * sizeof(Phys);
    q = reinterpret_cast<char *>((reinterpret_cast<uintptr_t>(q) + 63) & ~uintptr_t(63));
    e.d_norm = reinterpret_cast<double *>(q); q += n * sizeof(double);
    b->d_h0 = reinterpret_cast<double *>(q); q += n * sizeof(double);
    e.d_cyc = reinterpret_cast<int *>(q); q += n * sizeof(int);
    b->d_act = reinterpret_cast<int *>(q); q += n * sizeof(int);
    b->d_ndone = reinterpret_cast<int *>(q); q += n * sizeof(int);
    b->d_stat = reinterpret_cast<int *>(q); q += n * sizeof(int);
    e.d_rb = reinterpret_cast<int *>(q);
    std::vector<LevelDev> hV(nl);
    std::vector<Phys> hPH(n);
    for (int l = 0; l < e.nlev; ++l)
        for (int c = 0; c < n; ++c) hV[(size_t)l * n + c] = states[c]->lv[l];
    for (int c = 0; c < n; ++c) hPH[c] = states[c]->ph;
    if (hipMemcpy(dV, hV.data(), nl * sizeof(LevelDev), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dPH, hPH.data(), n * sizeof(Phys), hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(fail(FAS_EDEVICE, "batch descriptor upload failed"));
    if (hipHostMalloc(reinterpret_cast<void **>(&b->h_act), 2 * n * sizeof(int), hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(FAS_ENOMEM, "pinned allocation failed"));
    for (hipEvent_t &ev : b->ev_chunk)
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
            return cleanup(fail(FAS_EDEVICE, "event creation failed"));
    launch_fill_int(b->d_act, n, 1, e.st);
    launch_fill_int(e.d_rb, n, 0, e.st);
    // per level the first residual tile of each case (n + 1 entries), then
    // the cases by descending hyperplane-chain length (ni + nj) for the
    // sweep launches
    int *dtiles = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&dtiles), ((size_t)e.nlev * (n + 1) + n) * sizeof(int)) != hipSuccess)
        return cleanup(fail(FAS_ENOMEM, "batch allocation failed"));
    b->allocs.push_back(dtiles);
    std::vector<int> htiles((size_t)e.nlev * (n + 1) + n);
    int *horder = htiles.data() + (size_t)e.nlev * (n + 1);
    for (int c = 0; c < n; ++c) horder[c] = c;
    std::stable_sort(horder, horder + n, [&](int a, int b2) {
        const Lay &La = states[a]->lv[0].L, &Lb = states[b2]->lv[0].L;
        return La.ni + La.nj > Lb.ni + Lb.nj;
    });
    for (int l = 0; l < e.nlev; ++l) {
        std::vector<Lay> lays;
        for (int c = 0; c < n; ++c) lays.push_back(states[c]->lv[l].L);
        e.lev.push_back(make_blev(lays, dV + (size_t)l * n, dPH, b->d_act, e.d_cyc));
        int *t0 = htiles.data() + (size_t)l * (n + 1);
        t0[0] = 0;
        for (int c = 0; c < n; ++c) t0[c + 1] = t0[c] + residual_tiles(lays[c]);
        e.lev.back().k.tile0 = dtiles + (size_t)l * (n + 1);
        e.lev.back().k.order = dtiles + (size_t)e.nlev * (n + 1);
        e.lev.back().ntiles = t0[n];
    }
    if (hipMemcpy(dtiles, htiles.data(), htiles.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(fail(FAS_EDEVICE, "batch descriptor upload failed"));
    // autotuner: per level, the fastest sweep configuration that covers the
    // tallest grid (banded ones with 2 to 16 bands), timed on the batch itself
    if (autotune) {
        for (int l = 0; l < e.nlev; ++l) {
            const int need = e.lev[l].max_nj;
            int best = -1;
            float best_ms = 0.0f;
            for (int cfg = 0; cfg < sweep_cfg_count(); ++cfg) {
                const int rows = sweep_cfg_rows(cfg, need);
                if (rows < need) continue;
                if (sweep_cfg_banded(cfg)) {
                    const int nb = sweep_cfg_bands(cfg, need);
                    if (nb < 2 || nb > 16) continue;
                } else if (rows > 4 * std::max(need, 16)) {
                    continue;
                }
                float ms = 0.0f;
                fas_status st = time_sweep(e, l, cfg, 3, &ms);
                if (st != FAS_OK) return cleanup(st);
                if (best < 0 || ms < best_ms) {
                    best = cfg;
                    best_ms = ms;
                }
            }
            e.lev[l].sweep_cfg = best;
        }
    }
    if (hipStreamSynchronize(e.st) != hipSuccess) return cleanup(fail(FAS_EDEVICE, "batch set-up failed"));
    *out = b;
    return FAS_OK;
}

// the group holding the batch's tallest grid of a level
static fas_batch tallest_part(fas_batch b, int level) {
    fas_batch t = b->parts[0];
    for (fas_batch p : b->parts)
        if (p->e.lev[level].max_nj > t->e.lev[level].max_nj) t = p;
    return t;
}

extern "C" fas_status fas_batch_sweep_config(fas_batch b, int32_t level, int32_t *cfg, int32_t *rows) {
    if (!b || level < 0 || level >= b->e.nlev) return fail(FAS_EINVAL, "bad argument");
    if (!b->parts.empty()) return fas_batch_sweep_config(tallest_part(b, level), level, cfg, rows);
    int c = b->e.lev[level].sweep_cfg;
    if (c < 0) c = sweep_cfg_default(b->e.lev[level].max_nj, b->e.fp32);
    if (cfg) *cfg = c;
    if (rows) *rows = sweep_cfg_rows(c, b->e.lev[level].max_nj);
    return FAS_OK;
}

extern "C" int32_t fas_sweep_config_count(void) { return sweep_cfg_count(); }

extern "C" fas_status fas_sweep_config_info(int32_t cfg, int32_t *kind, int32_t *threads,
                                            int32_t *rows_per_workgroup, int32_t *depth_fp64,
                                            int32_t *depth_fp32) {
    if (cfg < 0 || cfg >= sweep_cfg_count() || !kind || !threads || !rows_per_workgroup || !depth_fp64 ||
        !depth_fp32)
        return fail(FAS_EINVAL, "bad argument");
    int k, t, r, a, b;
    sweep_cfg_info(cfg, &k, &t, &r, &a, &b);
    *kind = k;
    *threads = t;
    *rows_per_workgroup = r;
    *depth_fp64 = a;
    *depth_fp32 = b;
    return FAS_OK;
}

extern "C" fas_status fas_batch_set_sweep_config(fas_batch b, int32_t level, int32_t cfg) {
    if (!b || level < 0 || level >= b->e.nlev) return fail(FAS_EINVAL, "bad argument");
    if (!b->parts.empty()) {
        // checked against the tallest grid first, so no group is changed on a refusal
        STCHK(fas_batch_set_sweep_config(tallest_part(b, level), level, cfg));
        for (fas_batch p : b->parts) STCHK(fas_batch_set_sweep_config(p, level, cfg));
        return FAS_OK;
    }
    if (cfg < -1 || cfg >= sweep_cfg_count()) return fail(FAS_EINVAL, "bad sweep configuration");
    if (cfg >= 0 && sweep_cfg_rows(cfg, b->e.lev[level].max_nj) < b->e.lev[level].max_nj)
        return fail(FAS_EINVAL, "sweep configuration covers fewer rows than the tallest grid");
    b->e.lev[level].sweep_cfg = cfg;
    drop_graph(b);
    return FAS_OK;
}

// Start of a solve on one group: history rows, control record, every case
// active, the norm before the first cycle, and (use_graph) the captured
// cycle.
static fas_status batch_begin(fas_batch b, int32_t max_cycles, double drop_orders, int32_t use_graph,
                              BatchCtl &ctl) {
    Engine &e = b->e;
    const int n = e.n;
    if (max_cycles + 1 > b->hcap) {
        drop_graph(b);
        HIPCHK(hipStreamSynchronize(e.st));
        if (b->d_hist) {
            (void)hipFree(b->d_hist);
            for (auto &p : b->allocs)
                if (p == b->d_hist) p = nullptr;
        }
        b->d_hist = nullptr;
        HIPCHK(hipMalloc(&b->d_hist, (size_t)n * (max_cycles + 1) * sizeof(double)));
        b->allocs.push_back(b->d_hist);
        b->hcap = max_cycles + 1;
    }
    ctl = make_ctl(e, b->d_h0, b->d_hist, b->hcap, b->d_act, b->d_ndone, b->d_stat, max_cycles, drop_orders);
    // every case starts active; its c* ramp continues from its own count
    launch_fill_int(b->d_act, n, 1, e.st);
    for (int c = 0; c < n; ++c)
        HIPCHK(hipMemcpyAsync(e.d_cyc + c, b->states[c]->e.d_cyc, sizeof(int), hipMemcpyDeviceToDevice, e.st));
    e.has_src[0] = 0;
    eval_norm(e);
    launch_batch_init(ctl, n, e.st);
    HIPCHK(hipGetLastError());
    if (use_graph && (b->graph_cap != max_cycles || b->graph_drop != drop_orders)) {
        drop_graph(b);
        const int prof = e.prof;
        e.prof = 0;
        HIPCHK(hipStreamBeginCapture(e.st, hipStreamCaptureModeThreadLocal));
        controlled_cycle(e, ctl);
        hipError_t er = hipStreamEndCapture(e.st, &b->graph);
        e.prof = prof;
        if (er != hipSuccess) return fail(FAS_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(er));
        HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->graph_cap = max_cycles;
        b->graph_drop = drop_orders;
    }
    return FAS_OK;
}

static fas_status batch_cycle(fas_batch b, const BatchCtl &ctl, int32_t use_graph) {
    if (use_graph) HIPCHK(hipGraphLaunch(b->exec, b->e.st));
    else controlled_cycle(b->e, ctl);
    return FAS_OK;
}

// End of a solve on one group (its stream synchronised): cycle counts back
// to the states, per-case counts, status and history rows (row pitch
// max_cycles + 1), diverged cases' hand-off arrays re-armed.
static fas_status batch_collect(fas_batch b, int32_t max_cycles, int *nd, int *stv, double *res_hist) {
    Engine &e = b->e;
    const int n = e.n;
    for (int c = 0; c < n; ++c)
        HIPCHK(hipMemcpyAsync(b->states[c]->e.d_cyc, e.d_cyc + c, sizeof(int), hipMemcpyDeviceToDevice, e.st));
    HIPCHK(hipMemcpyAsync(nd, b->d_ndone, n * sizeof(int), hipMemcpyDeviceToHost, e.st));
    HIPCHK(hipMemcpyAsync(stv, b->d_stat, n * sizeof(int), hipMemcpyDeviceToHost, e.st));
    // a case's history is a row of hcap values (hcap can exceed this
    // solve's max_cycles + 1 after a longer solve)
    if (res_hist)
        HIPCHK(hipMemcpy2DAsync(res_hist, (size_t)(max_cycles + 1) * sizeof(double), b->d_hist,
                                (size_t)b->hcap * sizeof(double), (size_t)(max_cycles + 1) * sizeof(double), n,
                                hipMemcpyDeviceToHost, e.st));
    HIPCHK(hipStreamSynchronize(e.st));
    for (int c = 0; c < n; ++c)
        if (stv[c] == FAS_DIVERGED) rearm_handoff(b->states[c]->lv, e.st);
    HIPCHK(hipStreamSynchronize(e.st));
    return FAS_OK;
}

// worst status: diverged, stalled, not converged, ok
static int status_rank(int st) {
    return st == FAS_DIVERGED ? 3 : st == FAS_STALLED ? 2 : st == FAS_NOT_CONVERGED ? 1 : 0;
}

// Groups run concurrently, each replaying its own cycles on its own stream:
// the host keeps up to two chunks of CHECK cycles queued per group, each
// followed by an asynchronous copy of the group's activity flags, and polls
// the chunks' events; a group stops once a snapshot shows no active case or
// its cycles reach max_cycles.  Replays queued after a group's last case
// stopped are no-ops (the device flags mask them), so every case's iterates
// are those of a solve on its own.
static fas_status grouped_solve(fas_batch b, int32_t max_cycles, double drop_orders, int32_t use_graph,
                                int32_t *n_done, int32_t *status, double *res_hist) {
    const int G = (int)b->parts.size();
    constexpr int CHECK = 4;
    struct Run {
        BatchCtl ctl;
        int launched = 0, queued = 0, head = 0;
        bool done = false;
        hipEvent_t ev[2] = {nullptr, nullptr};
        int *snap[2] = {nullptr, nullptr};
    };
    std::vector<Run> runs(G);
    fas_status st = FAS_OK;
    int off = 0;
    for (int g = 0; g < G && st == FAS_OK; ++g) {
        Run &r = runs[g];
        const int m = b->parts[g]->e.n;
        r.snap[0] = b->h_flags + 2 * off;
        r.snap[1] = b->h_flags + 2 * off + m;
        off += m;
        for (int k = 0; k < 2; ++k)
            if (hipEventCreateWithFlags(&r.ev[k], hipEventDisableTiming) != hipSuccess)
                st = fail(FAS_EDEVICE, "event creation failed");
    }
    // the groups start after the work already queued on the batch stream
    if (st == FAS_OK && hipEventRecord(b->ev_start, b->e.st) != hipSuccess) st = fail(FAS_EDEVICE, "event record failed");
    for (int g = 0; g < G && st == FAS_OK; ++g) {
        if (hipStreamWaitEvent(b->parts[g]->e.st, b->ev_start, 0) != hipSuccess)
            st = fail(FAS_EDEVICE, "stream wait failed");
        else
            st = batch_begin(b->parts[g], max_cycles, drop_orders, use_graph, runs[g].ctl);
    }
    while (st == FAS_OK) {
        bool all = true;
        for (int g = 0; g < G && st == FAS_OK; ++g) {
            Run &r = runs[g];
            fas_batch p = b->parts[g];
            if (r.done) continue;
            all = false;
            if (r.queued > 0) {
                const hipError_t q = hipEventQuery(r.ev[r.head]);
                if (q == hipSuccess) {
                    int any = 0;
                    for (int c = 0; c < p->e.n; ++c) any |= r.snap[r.head][c];
                    r.head ^= 1;
                    --r.queued;
                    if (!any) {
                        r.done = true;
                        continue;
                    }
                } else if (q != hipErrorNotReady) {
                    st = fail(FAS_EDEVICE, std::string("cycle replay failed: ") + hipGetErrorString(q));
                    break;
                }
            }
            if (r.queued < 2 && r.launched < max_cycles) {
                const int k = std::min(CHECK, max_cycles - r.launched);
                for (int i = 0; i < k && st == FAS_OK; ++i) st = batch_cycle(p, r.ctl, use_graph);
                r.launched += k;
                const int slot = (r.head + r.queued) & 1;
                if (st == FAS_OK &&
                    (hipMemcpyAsync(r.snap[slot], p->d_act, p->e.n * sizeof(int), hipMemcpyDeviceToHost, p->e.st) !=
                         hipSuccess ||
                     hipEventRecord(r.ev[slot], p->e.st) != hipSuccess))
                    st = fail(FAS_EDEVICE, "cycle replay failed");
                ++r.queued;
            } else if (r.queued == 0 && r.launched >= max_cycles) {
                r.done = true;
            }
        }
        if (all) break;
        std::this_thread::yield();
    }
    // gather every group's results into the batch's case order
    int worst = FAS_OK;
    for (int g = 0; g < G; ++g) {
        fas_batch p = b->parts[g];
        const int m = p->e.n;
        if (hipStreamSynchronize(p->e.st) != hipSuccess && st == FAS_OK) st = fail(FAS_EDEVICE, "batch solve failed");
        if (st == FAS_OK) {
            std::vector<int> nd(m), stv(m);
            std::vector<double> h(res_hist ? (size_t)m * (max_cycles + 1) : 0);
            st = batch_collect(p, max_cycles, nd.data(), stv.data(), res_hist ? h.data() : nullptr);
            for (int k = 0; k < m && st == FAS_OK; ++k) {
                const int c = b->part_cases[g][k];
                if (n_done) n_done[c] = nd[k];
                if (status) status[c] = stv[k];
                if (status_rank(stv[k]) > status_rank(worst)) worst = stv[k];
                if (res_hist)
                    std::memcpy(res_hist + (size_t)c * (max_cycles + 1), h.data() + (size_t)k * (max_cycles + 1),
                                (size_t)(max_cycles + 1) * sizeof(double));
            }
        }
        for (int k = 0; k < 2; ++k)
            if (runs[g].ev[k]) (void)hipEventDestroy(runs[g].ev[k]);
    }
    if (st != FAS_OK) return st;
    if (worst != FAS_OK) g_err = std::string("batched case: ") + status_message(worst);
    return (fas_status)worst;
}

extern "C" fas_status fas_batch_solve(fas_batch b, int32_t max_cycles, double drop_orders, int32_t use_graph,
                                      int32_t *n_done, int32_t *status, double *res_hist) {
    if (!b || max_cycles < 0) return fail(FAS_EINVAL, "bad argument");
    if (!b->parts.empty()) return grouped_solve(b, max_cycles, drop_orders, use_graph, n_done, status, res_hist);
    Engine &e = b->e;
    const int n = e.n;
    BatchCtl ctl;
    STCHK(batch_begin(b, max_cycles, drop_orders, use_graph, ctl));
    STCHK(replay_chunks(e.st, max_cycles, b->d_act, n, b->h_act, b->ev_chunk,
                        [&]() { return batch_cycle(b, ctl, use_graph); }));
    std::vector<int> nd(n), stv(n);
    STCHK(batch_collect(b, max_cycles, nd.data(), stv.data(), res_hist));
    int worst = FAS_OK;
    for (int c = 0; c < n; ++c) {
        if (n_done) n_done[c] = nd[c];
        if (status) status[c] = stv[c];
        if (status_rank(stv[c]) > status_rank(worst)) worst = stv[c];
    }
    if (worst != FAS_OK) g_err = std::string("batched case: ") + status_message(worst);
    return (fas_status)worst;
}

extern "C" fas_status fas_batch_profile(fas_batch b, int32_t enable) {
    if (!b) return fail(FAS_EINVAL, "null batch");
    for (fas_batch p : b->parts) STCHK(profile_on(p->e, enable));
    if (!b->parts.empty()) return FAS_OK;
    return profile_on(b->e, enable);
}

extern "C" fas_status fas_batch_profile_read(fas_batch b, double *ms, int64_t *count) {
    if (!b) return fail(FAS_EINVAL, "null batch");
    if (b->parts.empty()) return profile_read(b->e, ms, count);
    // summed over the groups (concurrent groups overlap in time)
    for (int k = 0; k < FAS_PROF_NCLASS; ++k) {
        if (ms) ms[k] = 0.0;
        if (count) count[k] = 0;
    }
    for (fas_batch p : b->parts) {
        double pm[FAS_PROF_NCLASS];
        int64_t pc[FAS_PROF_NCLASS];
        STCHK(profile_read(p->e, pm, pc));
        for (int k = 0; k < FAS_PROF_NCLASS; ++k) {
            if (ms) ms[k] += pm[k];
            if (count) count[k] += pc[k];
        }
    }
    return FAS_OK;
}

extern "C" int64_t fas_set_four_lane_limit(int64_t max_cells) { return set_four_lane_limit(max_cells); }

extern "C" const char *fas_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------- discrete Fourier analysis
// descriptors of fas_dfa's cases into h (n_cases entries); *total = pairs
static fas_status dfa_descriptors(const fas_dfa_case *cases, int32_t n_cases, DfaCase *h, long long *total_out) {
    long long total = 0;
    for (int k = 0; k < n_cases; ++k) {
        const fas_dfa_case &c = cases[k];
        const double rho = c.u[0];
        const double p = (1.4 - 1.0) * (c.u[3] - 0.5 * (c.u[1] * c.u[1] + c.u[2] * c.u[2]) / rho);
        if (c.scheme < 0 || c.scheme > FAS_PARK51 || c.nx < 2 || c.ny < 2 || (c.nx & 1) || (c.ny & 1) ||
            !(rho > 0.0) || !(p > 0.0) || !(c.cstar > 0.0) || !(c.d >= 0.0) || !(c.ar > 0.0) ||
            !(c.eta > 0.0) || (c.unsteady && !(c.c > 0.0)) || !std::isfinite(c.cstar) || !std::isfinite(c.c) ||
            c.precond < FAS_DFA_SGS || c.precond > FAS_DFA_NONE || (c.unsplit != 0 && c.unsplit != 1) ||
            (c.mesh != FAS_DFA_MESH_AR_DX && c.mesh != FAS_DFA_MESH_DX_OVER_AR))
            return fail(FAS_EINVAL, "bad Fourier analysis case");
        const Scheme &sc = SCHEMES[c.scheme];
        DfaCase &d = h[k];
        std::memset(&d, 0, sizeof(d));
        for (int q = 0; q < 4; ++q) d.u[q] = c.u[q];
        for (int q = 0; q < sc.s; ++q) {
            d.alpha[q] = sc.alpha[q];
            d.beta[q] = c.unsplit ? 1.0 : sc.beta[q];
        }
        d.precond = c.precond;
        d.mesh = c.mesh;
        d.s = sc.s;
        d.wform = sc.aw;
        d.nx = c.nx;
        d.ny = c.ny;
        d.unsteady = c.unsteady ? 1 : 0;
        d.cstar = c.cstar;
        d.d = c.d;
        d.eta = c.eta;
        d.ar = c.ar;
        d.c = c.c;
        d.start = total;
        total += (long long)c.nx * c.ny;
    }
    if (total > (1ll << 31)) return fail(FAS_EINVAL, "too many phase angles");
    *total_out = total;
    return FAS_OK;
}

// upload the descriptors to dc, run the analysis, wait for the results
static fas_status dfa_run(const DfaCase *h, DfaCase *dc, int32_t n_cases, long long total, double *amp,
                          double *smooth, double *radius, hipStream_t st) {
    if (hipMemcpyAsync(dc, h, (size_t)n_cases * sizeof(DfaCase), hipMemcpyHostToDevice, st) != hipSuccess)
        return fail(FAS_EDEVICE, "descriptor upload failed");
    launch_dfa(dc, n_cases, total, radius, amp, smooth, st);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
        return fail(FAS_EDEVICE, "Fourier analysis kernel failed");
    return FAS_OK;
}

extern "C" fas_status fas_dfa(const fas_dfa_case *cases, int32_t n_cases, double *amp, double *smooth,
                              double *radius, void *stream) {
    if (!cases || n_cases <= 0 || !amp || !smooth) return fail(FAS_EINVAL, "bad argument");
    std::vector<DfaCase> h(n_cases);
    long long total = 0;
    STCHK(dfa_descriptors(cases, n_cases, h.data(), &total));
    hipStream_t st = (hipStream_t)stream;
    DfaCase *dc = nullptr;
    HIPCHK(hipMalloc(&dc, h.size() * sizeof(DfaCase)));
    const fas_status out = dfa_run(h.data(), dc, n_cases, total, amp, smooth, radius, st);
    (void)hipFree(dc);
    return out;
}

// Allocation-free variant of fas_dfa: the descriptor table lives in a
// file-scope device array (each GPU holds its own copy for the life of the
// process); its address on each device is looked up once, with that device
// current, and the host staging table is a static array.  A mutex
// serialises the library's own calls up to the point where the results are
// written.
static __device__ __align__(256) DfaCase scratch[FAS_DFA_NOALLOC_MAX_CASES];
static DfaCase g_dfa_host[FAS_DFA_NOALLOC_MAX_CASES];
static std::mutex g_dfa_mutex;
constexpr int MAX_DEVICES = 64;
static DfaCase *g_scratch_ptr[MAX_DEVICES] = {nullptr};

extern "C" fas_status fas_dfa_noalloc(const fas_dfa_case *cases, int32_t n_cases, double *amp, double *smooth,
                                      double *radius, void *stream) {
    if (!cases || n_cases <= 0 || !amp || !smooth) return fail(FAS_EINVAL, "bad argument");
    if (n_cases > FAS_DFA_NOALLOC_MAX_CASES)
        return fail(FAS_EINVAL, "more cases than the allocation-free table holds (FAS_DFA_NOALLOC_MAX_CASES)");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(FAS_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_dfa_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = static_cast<DfaCase *>(ptr);
    }
    long long total = 0;
    STCHK(dfa_descriptors(cases, n_cases, g_dfa_host, &total));
    return dfa_run(g_dfa_host, g_scratch_ptr[dev], n_cases, total, amp, smooth, radius, (hipStream_t)stream);
}

