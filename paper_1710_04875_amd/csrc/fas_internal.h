// Internal data layout of the MI355X FAS library (not part of the ABI).
//
// Every per-cell array of a level lives in one "skewed" padded layout: the
// interior ni x nj cells plus two ghost layers on every side (NI = ni + 4,
// NJ = nj + 4 padded cells), cell (I, J) of the padded grid stored at slot
//     s = (I + J) * NJ + J.
// Cells of one hyperplane I + J = const are contiguous, so the
// Gauss-Seidel wavefront (one sweep row per thread, all rows advancing one
// hyperplane per step) reads and writes coalesced lines, and every
// stencil neighbour is a constant slot offset:
//     (I+1, J) = +NJ,  (I, J+1) = +NJ+1,  (I+1, J-1) = -1,  (I-1, J+1) = +1.
// Arrays are planes of NS = (NI + NJ - 1) * NJ values, one plane per
// component.  Slots outside the padded rectangle are never read.
//
// Every kernel of the cycle works on a batch of independent cases: it
// receives a device array of per-case level descriptors (LevelDev) and
// per-case physics (Phys), takes its case from a block index, and skips
// cases whose activity flag is 0.  A single flow state is a batch of one.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace fas {

constexpr double GAM = 1.4;
constexpr int NG = 2;

struct Lay {
    int ni, nj, NI, NJ, NS, nw, topo;
    __host__ __device__ int slot(int i, int j) const { return (i + j + 2 * NG) * NJ + (j + NG); }
};

// geometry planes (all padded cells unless noted)
enum GeoPlane {
    G_SXI_X, G_SXI_Y,     // west face vector of cell (i in [0,ni], j interior)
    G_SETA_X, G_SETA_Y,   // south face vector (i interior, j in [0,nj])
    G_SB0, G_SB1, G_SB2, G_SB3,  // mean i- and j- face vectors
    G_VOL, G_XC, G_YC,    // volume, centre
    G_WD,                 // distance to the j = 0 face (fine level, interior)
    G_WIX, G_WIY,         // moving mesh: grid velocity at the midpoint of i-face (I, j)
    G_WJX, G_WJY,         // moving mesh: grid velocity at the midpoint of j-face (i, J)
    G_NPLANES
};

// per-cell quantity planes recomputed for every residual evaluation
enum CqPlane { Q_P, Q_Q, Q_RXI, Q_RETA, Q_T, Q_NPLANES };
// vertex-gradient planes, vertex (I, J) stored at the slot of cell (I, J)
enum VgPlane { V_UX, V_UY, V_VX, V_VY, V_TX, V_TY, V_NPLANES };

// preconditioner blocks: five 4x4 blocks per cell, D^-1 and M_s = D^-1 B_s
// for the four neighbour slots (0 west, 1 east, 2 south or wake-cut
// partner, 3 north).
constexpr int B_DINV = 0;
constexpr int B_M0 = 1;          // + slot
constexpr int BLK_NBLOCKS = 5;
constexpr int BLK_NPLANES = 80;  // values per cell

// Element (row r, column c) of block b of cell slot s.  FP32 blocks: one
// 16-value record per cell (a block row is one 16-byte vector).  FP64
// blocks: two half planes per block, columns 0-1 and 2-3, each holding the
// four rows' column pairs of a cell contiguously (64 bytes), so that the
// 16-byte loads of a wave reading one block row for consecutive cells form
// one contiguous run.
template <typename T> struct BL;
template <> struct BL<float> {
    __host__ __device__ static size_t at(int b, int NS, int s, int r, int c) {
        return ((size_t)b * NS + s) * 16 + r * 4 + c;
    }
};
template <> struct BL<double> {
    __host__ __device__ static size_t at(int b, int NS, int s, int r, int c) {
        return ((size_t)(2 * b + (c >> 1)) * NS + s) * 8 + r * 2 + (c & 1);
    }
};

struct Phys {
    double mach, alpha_deg, re, pr, prt, mu_inf;
    double uinf[4];
    double eta, d_cut, kappa2c;
    // pseudo-time step c*: cfl_ramp for n_ramp cycles, then growth by
    // ramp_growth per cycle up to cfl
    double cfl, cfl_ramp, ramp_growth;
    int n_ramp;
    int dt_form;      // 0: dt* = c* Omega / (r_xi + r_eta); 1: c* Omega / max(r_xi, r_eta)
    int rans;
    // rigidly rotating mesh (ALE): rate omega about (px, py); grid
    // velocities omega x (r - pivot) are in the G_W* planes
    int ale;
    double omega, px, py;
};

struct LevelDev {
    Lay L;
    double *geo;      // G_NPLANES * NS
    double *u;        // 4 * NS   current solution (ghosts filled on demand)
    double *u0;       // 4 * NS   solution at the start of a smoother iteration
    double *acc;      // 4 * NS   blended f^v accumulator
    double *F;        // 4 * NS   residual scratch (F_l(u) - s_l or F_l(u))
    double *src;      // 4 * NS   FAS source s_l (coarse levels)
    double *ut;       // 4 * NS   restricted solution u~ (coarse levels)
    double *un, *unm1;// 4 * NS   physical time levels
    double *ulast;    // 4 * NS   solution before the current cycle (roll-back of a diverged cycle)
    double *dts;      // NS
    double *mut;      // NS       eddy viscosity (fine: Baldwin-Lomax; coarse: restricted)
    double *cq;       // Q_NPLANES * NS
    double *vg;       // V_NPLANES * NS (RANS)
    void *blk;        // BLK_NPLANES * NS, double or float
    void *g;          // 4 * NS   D^-1 (dt* r) / forward sweep input
    void *y;          // 4 * NS   forward sweep output
    void *bnd;        // bnd_count(L) hand-off between row bands of one sweep (a sentinel
                      //          marks every slot not yet written in a launch)
    double *red;      // reduction scratch (RED_BLOCKS values)
};

// hand-off array of the banded sweeps: component r of row j on hyperplane
// h at ((r HB + h + BND_HOFF) NJ + j), for h in [-BND_HOFF, ni + nj +
// BND_HOFF), so that prefetches and padded steps stay inside their plane
constexpr int BND_HOFF = 32;
__host__ __device__ inline int bnd_hb(const Lay &L) { return L.ni + L.nj + 2 * BND_HOFF; }
__host__ __device__ inline size_t bnd_count(const Lay &L) { return (size_t)4 * bnd_hb(L) * L.NJ; }

// bit pattern of an unwritten hand-off slot: a signalling NaN in FP64 and,
// in each 32-bit half, a NaN payload no FP32 arithmetic produces
constexpr unsigned BND_SENTINEL32 = 0x7FF5A5A5u;
constexpr unsigned long long BND_SENTINEL64 = 0x7FF5A5A57FF5A5A5ull;

// 4-component vector fields of a level, addressed by name in batched
// launches (each case has its own pointers)
enum Field { FLD_U, FLD_U0, FLD_ACC, FLD_F, FLD_SRC, FLD_UT, FLD_UN, FLD_UNM1, FLD_ULAST, FLD_NONE };

__host__ __device__ inline double *field(const LevelDev &d, int f) {
    switch (f) {
        case FLD_U: return d.u;
        case FLD_U0: return d.u0;
        case FLD_ACC: return d.acc;
        case FLD_F: return d.F;
        case FLD_SRC: return d.src;
        case FLD_UT: return d.ut;
        case FLD_UN: return d.un;
        case FLD_UNM1: return d.unm1;
        case FLD_ULAST: return d.ulast;
        default: return nullptr;
    }
}

// device view of one level of a batch (kernel argument)
struct BK {
    const LevelDev *V;    // [n]
    const Phys *PH;       // [n]
    const int *act;       // [n] 0 = skip the case; nullptr = all active
    const int *cyc;       // [n] completed FAS cycles (c* ramp)
    const int *tile0;     // [n + 1] first residual tile of each case (batches), nullptr for one state
    const int *order;     // [n] cases by descending chain length (sweep launches), nullptr: in turn
    int n;                // cases
};

// host descriptor of one level of a batch
struct BLev {
    BK k;
    int n;                // cases
    int max_ns, max_ni, max_nj, max_nw;   // launch sizing over the cases
    int sweep_cfg;        // sweep kernel configuration (-1: by max_nj)
    int ntiles;           // residual tiles of all cases (k.tile0[n])
};

// residual tiles of one grid (the tiled residual's launch unit)
int residual_tiles(const Lay &L);

// ---------------------------------------------------------------- launchers
// geometry (one grid, at creation)
void launch_geom_interior(const Lay &L, const double *xn, const double *yn, double *geo,
                          const double *vol_children, const Lay *Lf, const double *geo_f,
                          hipStream_t st);
void launch_geom_ghost(const Lay &L, const double *xn, const double *yn, double *geo, hipStream_t st);

// rigid rotation of a level's geometry by (c, s) = (cos, sin) of the
// angle about (px, py), grid velocities for the rate omega
void launch_rotate_geometry(const Lay &L, const double *geo_ref, const double *xn, const double *yn,
                            double *geo, double c, double s, double px, double py, double omega,
                            hipStream_t st);

// residual chain
void launch_ghost_cq(const BLev &B, int noslip, int rans, hipStream_t st);   // both in one pass
void launch_vertex_gradients(const BLev &B, hipStream_t st);
void launch_baldwin_lomax(const BLev &B, hipStream_t st);
void launch_mut_ghosts(const BLev &B, hipStream_t st);

struct ResArgs {
    int fine;          // second-order JST (sensor, fourth difference)
    int viscous;       // add the viscous flux (RANS levels)
    int bdf;           // 0 steady, 1 implicit Euler, 2 BDF2
    double dt;         // physical time step
    int forcing;       // subtract src
    int mode;          // 0: write F = F^c + F^v, 1: smoother stage (acc, g)
    int stage;         // stage index (mode 1)
    double beta;       // beta_{i+1} of the blended f^v (stage > 0)
    int aw;            // 1: g = D^-1 (dt* r); 0: g = D^-1 r
    int fp32;          // blocks / g in float
    int src_acc;       // mode 0: also write src = F + acc (a coarse level's FAS forcing)
};
void launch_residual(const BLev &B, const ResArgs &a, hipStream_t st);

// preconditioner (the kernel also writes the level's dt*, Section 4.1, and
// on request copies u to u0, the smoother iteration's starting state)
void launch_blocks(const BLev &B, int aw, double tau, int viscous, int fp32, hipStream_t st, int copy_u0 = 0);
struct SweepArgs {
    int update;        // 1: write u = u0 - alpha x (AW) or u0 - alpha dt* x (pARK)
    double alpha;
    int aw;
    int xout_acc;      // 1: also write x (FP64) into the level's acc field
    int bands;         // row bands per case of a banded launch (set by the launcher)
};
void launch_sgs(const BLev &B, const SweepArgs &a, int fp32, hipStream_t st);
void launch_dinv(const BLev &B, int fp32, hipStream_t st);   // g = D^-1 F

// sweep kernel configurations for the autotuner: cfg indexes a table of
// (threads, rows per 4-thread group, prefetch depth); -1 picks by nj
int sweep_cfg_count();
int sweep_cfg_bands(int cfg, int max_nj);  // workgroups per case (1 unless banded)
int sweep_cfg_rows(int cfg, int max_nj);   // rows one launch covers per case
bool sweep_cfg_banded(int cfg);
void sweep_cfg_info(int cfg, int *kind, int *threads, int *rows, int *d64, int *d32);
int sweep_cfg_default(int max_nj, int fp32);
int sweep_cfg_plain(int max_nj);

// transfers and utilities
void launch_restrict(const BLev &Bf, const BLev &Bc, int fin, int fout, int fout2, hipStream_t st);
// restriction of up to two fine-level combinations a x (+ b y) in one launch
struct RJob {
    int fx;
    double a;
    int fy;            // FLD_NONE: a x alone
    double b;
    int fout, fout2;   // coarse outputs (fout2 may be FLD_NONE)
};
// (mut: also the volume-weighted eddy viscosity)
void launch_restrict_jobs(const BLev &Bf, const BLev &Bc, const RJob *jobs, int njobs, int mut, hipStream_t st);
void launch_prolong(const BLev &Bf, const BLev &Bc, hipStream_t st);
void launch_axpby(const BLev &B, double a, int fx, double b, int fy, int fout, hipStream_t st);
void launch_pack(const Lay &L, const double *padded, double *natural, int ncomp, hipStream_t st);
void launch_unpack(const Lay &L, const double *natural, double *padded, int ncomp, hipStream_t st);
void launch_norm(const BLev &B, double *out, hipStream_t st);   // out[n]
void launch_count_cycle(const BLev &B, int *cyc, hipStream_t st);
void launch_fill_int(int *p, int n, int v, hipStream_t st);
int norm_scratch_size();

// discrete adjoint of the steady fine-level residual (frozen eddy viscosity)
// out += (dF/du)^T lam (part 0), (df^c/du)^T lam (1) or (df^v/du)^T lam (2)
void launch_vjp(const Lay &L, const double *geo, const double *u, const double *mut, const Phys &ph,
                const double *lam, double *out, hipStream_t st, int part = 0);
void launch_param_partials(const Lay &L, const double *geo, const double *u, const double *mut,
                           const Phys &ph, double reynolds, double *dFa, double *dFm, hipStream_t st);
// grid-node sensitivities: gbar (metric planes G_SXI_X .. G_YC, zeroed)
// += (dF/dG)^T lam; gbar += dC_L/dG of the wall faces; dx, dy (zeroed node
// arrays) += (dG/dX)^T gbar
void launch_vjp_geo(const Lay &L, const double *geo, const double *u, const double *mut, const Phys &ph,
                    const double *lam, double *gbar, hipStream_t st);
void launch_forces_geo(const Lay &L, const double *geo, const double *u, const Phys &ph, double *gbar,
                       hipStream_t st);
void launch_geo_nodes(const Lay &L, const double *xn, const double *yn, const double *gbar, double *dx,
                      double *dy, hipStream_t st);
void launch_forces(const Lay &L, const double *geo, const double *u, const Phys &ph, double *out,
                   double *dcl, hipStream_t st);                       // out[6], dcl padded (zeroed)
// transposed SGS solve through the primal sweep: bt = the neighbour blocks
// transposed into the slots of the cells they act on, g = r in the sweep
// precision, and x = D^-T xi after the sweep
void launch_blocks_t(const Lay &L, const void *blk, void *bt, int fp32, hipStream_t st);
void launch_to_sweep(const Lay &L, const double *r, void *g, int fp32, hipStream_t st);
void launch_dinv_t(const Lay &L, const void *blk, const double *xi, double *x, int fp32, hipStream_t st);
int dot_scratch_size();
void launch_dot(const Lay &L, const double *a, const double *b, double *red, double *out, hipStream_t st);
void launch_axpby_ptr(const Lay &L, double a, const double *x, double b, const double *y, double *out,
                      hipStream_t st);
// lc += P^T lf (P: bilinear prolongation from Lc to Lf); lf += R^T lc (R:
// volume-weighted agglomeration from Lf to Lc)
void launch_adj_prolong_t(const Lay &Lf, const Lay &Lc, const double *lf, double *lc, hipStream_t st);
void launch_adj_restrict_t(const Lay &Lf, const Lay &Lc, const double *geof, const double *geoc, const double *lc,
                           double *lf, hipStream_t st);
void launch_adj_update(const Lay &L, const double *x, double a, const double *dts, const double *z,
                       double *out, hipStream_t st);
void launch_zero(double *p, size_t n, hipStream_t st);
// out[i] = <w, basis_i>, i < n (red: n * dot_scratch_size() values); w -= sum h_i basis_i
void launch_mdot(const Lay &L, const double *w, const double *basis, size_t V, int n, double *red,
                 double *out, hipStream_t st);
void launch_maxpy(const Lay &L, double *w, const double *basis, size_t V, const double *h, int n,
                  hipStream_t st);

// batch convergence control: per case c, after the norm of a cycle
struct BatchCtl {
    const double *nrm;    // [n] norm after the cycle
    double *h0;           // [n] norm before the first cycle
    double *hist;         // [n * hcap]
    int hcap;
    int *act, *cyc, *ndone, *stat;
    double drop_factor;   // 10^-drop (0: run to max_cycles)
    int max_cycles;
    int stall_window;     // > 0: stall test over this many cycles
    double stall_factor;  // 10^-stall_orders
    double growth_limit;  // > 0: a norm above growth_limit h0 is divergence
    int *rb;              // [n] 1: the case diverged in this cycle (roll back its solution)
};
// status of the stall test (fas_status value)
constexpr int ST_STALLED_CODE = -5;
void launch_batch_init(const BatchCtl &c, int n, hipStream_t st);
void launch_batch_status(const BatchCtl &c, int n, hipStream_t st);
// fine level: ulast = u for the active cases (before a cycle); u = ulast
// for the cases whose flag rb is set (after the status update)
void launch_save_u(const BLev &B, hipStream_t st);
void launch_rollback(const BLev &B, const int *rb, hipStream_t st);
// four-lane residual / block kernels up to this many cells per launch
long long four_lane_limit();
long long set_four_lane_limit(long long cells);

}  // namespace fas
