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
    G_NPLANES
};

// per-cell quantity planes recomputed for every residual evaluation
enum CqPlane { Q_P, Q_Q, Q_RXI, Q_RETA, Q_T, Q_NPLANES };
// vertex-gradient planes, vertex (I, J) stored at the slot of cell (I, J)
enum VgPlane { V_UX, V_UY, V_VX, V_VY, V_TX, V_TY, V_NPLANES };

// preconditioner blocks: five 4x4 blocks per cell, D^-1 and M_s = D^-1 B_s
// for the four neighbour slots (0 west, 1 east, 2 south or wake-cut
// partner, 3 north).  Block b of cell slot s is a contiguous row-major
// record of 16 values at (b * NS + s) * 16, so one row of a block is one
// aligned 4-vector and a wave reading rows of consecutive cells reads one
// contiguous run.
constexpr int B_DINV = 0;
constexpr int B_M0 = 1;          // + slot
constexpr int BLK_NBLOCKS = 5;
constexpr int BLK_NPLANES = 80;  // values per cell

struct Phys {
    double mach, alpha_deg, re, pr, prt, mu_inf;
    double uinf[4];
    double eta, d_cut, kappa2c;
    int rans;
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
    double *dts;      // NS
    double *mut;      // NS       eddy viscosity (fine level)
    double *cq;       // Q_NPLANES * NS
    double *vg;       // V_NPLANES * NS (fine RANS)
    void *blk;        // BLK_NPLANES * NS, double or float
    void *g;          // 4 * NS   D^-1 (dt* r) / forward sweep input
    void *y;          // 4 * NS   forward sweep output
    double *red;      // reduction scratch
};

// ---------------------------------------------------------------- launchers
// geometry
void launch_geom_interior(const Lay &L, const double *xn, const double *yn, double *geo,
                          const double *vol_children, const Lay *Lf, const double *geo_f,
                          hipStream_t st);
void launch_geom_ghost(const Lay &L, const double *xn, const double *yn, double *geo, hipStream_t st);

// residual chain
void launch_ghost_state(const Lay &L, const double *geo, double *u, const Phys &ph, int noslip,
                        hipStream_t st);
void launch_cell_quantities(const Lay &L, const double *geo, const double *u, double *cq, int rans,
                            hipStream_t st);
void launch_vertex_gradients(const Lay &L, const double *geo, const double *u, const double *cq,
                             double *vg, hipStream_t st);
void launch_baldwin_lomax(const Lay &L, const double *geo, const double *u, const double *cq,
                          const double *vg, double *mut, const Phys &ph, hipStream_t st);
void launch_mut_ghosts(const Lay &L, double *mut, hipStream_t st);
void launch_local_time_step(const Lay &L, const double *geo, const double *u, double *dts,
                            double cfl, hipStream_t st);

struct ResArgs {
    int fine;          // second-order JST (sensor, fourth difference)
    int viscous;       // add the viscous flux (fine RANS)
    int bdf;           // 0 steady, 1 implicit Euler, 2 BDF2
    double dt;         // physical time step
    int forcing;       // subtract src
    int mode;          // 0: write F = F^c + F^v, 1: smoother stage (acc, g)
    int stage;         // stage index (mode 1)
    double beta;       // beta_{i+1} of the blended f^v (stage > 0)
    int aw;            // 1: g = D^-1 (dt* r); 0: g = D^-1 r
    int fp32;          // blocks / g in float
};
void launch_residual(const Lay &L, const double *geo, const double *u, const double *cq,
                     const double *vg, const double *mut, const double *un, const double *unm1,
                     const double *src, const Phys &ph, const ResArgs &a, double *F, double *acc,
                     const double *dts, const void *blk, void *g, hipStream_t st);

// preconditioner
void launch_blocks(const Lay &L, const double *geo, const double *u, const double *cq,
                   const double *mut, const double *dts, const Phys &ph, int aw, double tau,
                   int viscous, int fp32, void *blk, hipStream_t st);
struct SweepArgs {
    int update;        // 1: write u = u0 - alpha x (AW) or u0 - alpha dt* x (pARK)
    double alpha;
    int aw;
    double *u;         // padded solution to update
    const double *u0;
    const double *dts;
    double *xout;      // optional: x written here (padded, 4 planes)
};
void launch_sgs(const Lay &L, const void *blk, const void *g, void *y, const SweepArgs &a,
                int fp32, hipStream_t st);

// transfers and utilities
void launch_restrict(const Lay &Lf, const Lay &Lc, const double *geo_f, const double *geo_c,
                     const double *vf, double *vc, double *vc_copy, hipStream_t st);
void launch_prolong(const Lay &Lf, const Lay &Lc, const double *uc, const double *utc, double *uf,
                    hipStream_t st);
void launch_axpby_interior(const Lay &L, double a, const double *x, double b, const double *y,
                           double *out, int ncomp, hipStream_t st);
void launch_pack(const Lay &L, const double *padded, double *natural, int ncomp, hipStream_t st);
void launch_unpack(const Lay &L, const double *natural, double *padded, int ncomp, hipStream_t st);
void launch_norm(const Lay &L, const double *F, double *red, double *out, hipStream_t st);
int norm_scratch_size(const Lay &L);

}  // namespace fas
