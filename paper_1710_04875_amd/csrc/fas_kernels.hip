// HIP kernels (gfx950) of the preconditioned FAS smoother.
//
// Paper: Birken, Bull, Jameson, "Preconditioned smoothers for the full
// approximation scheme for the RANS equations".  Each kernel names the
// section / equation it implements.  Layout: fas_internal.h.
#include "fas_internal.h"
#include "fas_geom.h"
#include "fas_cells.h"
#include "fas_dfa.h"

#include <cmath>
#include <type_traits>
#include <utility>

namespace fas {

namespace {

constexpr int TPB = 256;
constexpr double SUTH = 110.4 / 288.15;
constexpr double BL_APLUS = 26.0, BL_CCP = 1.6, BL_CKLEB = 0.3, BL_CWK = 0.25,
                 BL_KAPPA = 0.4, BL_K = 0.0168;

inline int nblocks(int n, int t = TPB) { return (n + t - 1) / t; }

__device__ inline bool decode(const Lay &L, int s, int &i, int &j) {
    if (s >= L.NS) return false;
    int H = s / L.NJ;
    int J = s - H * L.NJ;
    int I = H - J;
    if (I < 0 || I >= L.NI) return false;
    i = I - NG;
    j = J - NG;
    return true;
}

__device__ inline bool interior(const Lay &L, int i, int j) {
    return i >= 0 && i < L.ni && j >= 0 && j < L.nj;
}

__device__ inline bool cut_col(const Lay &L, int i) {
    return L.topo == 1 && (i < L.nw || i >= L.ni - L.nw);
}

__device__ inline double pres(double r, double mx, double my, double E) {
    return (GAM - 1.0) * (E - 0.5 * (mx * mx + my * my) / r);
}

__device__ inline double sutherland(double T, double mu_inf) {
    return ((mu_inf * (T * sqrt(T))) * (1.0 + SUTH)) / (T + SUTH);
}

__device__ inline size_t brec(int b, int NS, int s) { return ((size_t)b * NS + s) * 16; }


template <typename T> struct V4;
template <> struct V4<double> {
    __device__ static void load(const double *p, double o[4]) {
        double2 a = *reinterpret_cast<const double2 *>(p);
        double2 b = *reinterpret_cast<const double2 *>(p + 2);
        o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
    }
};
template <> struct V4<float> {
    __device__ static void load(const float *p, float o[4]) {
        float4 a = *reinterpret_cast<const float4 *>(p);
        o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
    }
};

// workgroup barrier that waits for LDS traffic only (global loads issued
// for later hyperplanes stay in flight across it)
__device__ inline void lds_barrier() {
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0), vmcnt / expcnt untouched
    __builtin_amdgcn_s_barrier();
}

__device__ inline void ld4(const double *a, int NS, int s, double v[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = a[k * NS + s];
}

// Pointers read from a descriptor in memory carry no address space, so the
// compiler would access them with flat instructions, which also count on
// the LDS wait counter (an LDS-only barrier would then drain every
// prefetch in flight).  The descriptor is therefore read through a mirror
// whose pointers are typed global, and every access derived from them
// becomes a global load or store.
#define FAS_GLOBAL __attribute__((address_space(1)))
struct LevelDevG {
    Lay L;
    FAS_GLOBAL double *geo, *u, *u0, *acc, *F, *src, *ut, *un, *unm1, *ulast, *dts, *mut, *cq, *vg;
    FAS_GLOBAL char *blk, *g, *y, *bnd;
    FAS_GLOBAL double *red;
};
static_assert(sizeof(LevelDevG) == sizeof(LevelDev), "descriptor mirror layout");

// the level descriptor of case c of a batched launch; false if the case is
// inactive (the whole block then returns before any barrier)
__device__ inline bool take(const BK &b, int c, LevelDev &d) {
    if (b.act != nullptr && b.act[c] == 0) return false;
    const LevelDevG &s = reinterpret_cast<const LevelDevG *>(b.V)[c];
    d.L = s.L;
    d.geo = (double *)s.geo;
    d.u = (double *)s.u;
    d.u0 = (double *)s.u0;
    d.acc = (double *)s.acc;
    d.F = (double *)s.F;
    d.src = (double *)s.src;
    d.ut = (double *)s.ut;
    d.un = (double *)s.un;
    d.unm1 = (double *)s.unm1;
    d.ulast = (double *)s.ulast;
    d.dts = (double *)s.dts;
    d.mut = (double *)s.mut;
    d.cq = (double *)s.cq;
    d.vg = (double *)s.vg;
    d.blk = (void *)s.blk;
    d.g = (void *)s.g;
    d.y = (void *)s.y;
    d.bnd = (void *)s.bnd;
    d.red = (double *)s.red;
    return true;
}

// ------------------------------------------------------------------ geometry
// Section 2 (finite volumes on a structured mesh), Section 3 (agglomerated
// coarse levels: coarse face = sum of child faces, coarse volume = sum of
// child volumes).
__global__ void k_geom_interior(Lay L, const double *xn, const double *yn, double *geo,
                                const double *volf, Lay Lf) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    int i, j;
    if (!decode(L, s, i, j)) return;
    const int NS = L.NS, W = L.ni + 1;
    auto X = [&](int I, int J) { return xn[J * W + I]; };
    auto Y = [&](int I, int J) { return yn[J * W + I]; };
    if (i >= 0 && i <= L.ni && j >= 0 && j < L.nj) {
        double sx, sy;
        g_iface<double>(X, Y, i, j, sx, sy);
        geo[G_SXI_X * NS + s] = sx;
        geo[G_SXI_Y * NS + s] = sy;
    }
    if (i >= 0 && i < L.ni && j >= 0 && j <= L.nj) {
        double sx, sy;
        g_jface<double>(X, Y, i, j, sx, sy);
        geo[G_SETA_X * NS + s] = sx;
        geo[G_SETA_Y * NS + s] = sy;
    }
    if (!interior(L, i, j)) return;
    double vol, xc, yc, sb[4];
    g_cell(X, Y, i, j, vol, xc, yc, sb);
    if (volf != nullptr) {
        double v00 = volf[Lf.slot(2 * i, 2 * j)], v10 = volf[Lf.slot(2 * i + 1, 2 * j)];
        double v01 = volf[Lf.slot(2 * i, 2 * j + 1)], v11 = volf[Lf.slot(2 * i + 1, 2 * j + 1)];
        vol = ((v00 + v10) + v01) + v11;
    }
    geo[G_VOL * NS + s] = vol;
    geo[G_XC * NS + s] = xc;
    geo[G_YC * NS + s] = yc;
    geo[G_SB0 * NS + s] = sb[0];
    geo[G_SB1 * NS + s] = sb[1];
    geo[G_SB2 * NS + s] = sb[2];
    geo[G_SB3 * NS + s] = sb[3];
    double mx = 0.5 * (X(i, 0) + X(i + 1, 0)), my = 0.5 * (Y(i, 0) + Y(i + 1, 0));
    double cx = xc - mx, cy = yc - my;
    geo[G_WD * NS + s] = sqrt(cx * cx + cy * cy);
}

// Rigid rotation of a level (moving mesh): vectors and points rotate by
// (c, s) about (px, py), volumes and wall distances are unchanged; grid
// velocities omega x (r - pivot) at the rotated face midpoints.
__global__ void k_rotate_geometry(Lay L, const double *geo0, const double *xn, const double *yn, double *geo,
                                  double c, double s, double px, double py, double omega) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    int i, j;
    if (!decode(L, t, i, j)) return;
    const int NS = L.NS, W = L.ni + 1;
    auto vec = [&](int px_, int py_) {
        const double vx = geo0[px_ * NS + t], vy = geo0[py_ * NS + t];
        geo[px_ * NS + t] = c * vx - s * vy;
        geo[py_ * NS + t] = s * vx + c * vy;
    };
    vec(G_SXI_X, G_SXI_Y);
    vec(G_SETA_X, G_SETA_Y);
    vec(G_SB0, G_SB1);
    vec(G_SB2, G_SB3);
    {
        const double dx = geo0[G_XC * NS + t] - px, dy = geo0[G_YC * NS + t] - py;
        geo[G_XC * NS + t] = px + (c * dx - s * dy);
        geo[G_YC * NS + t] = py + (s * dx + c * dy);
    }
    geo[G_VOL * NS + t] = geo0[G_VOL * NS + t];
    geo[G_WD * NS + t] = geo0[G_WD * NS + t];
    double wix = 0.0, wiy = 0.0, wjx = 0.0, wjy = 0.0;
    if (i >= 0 && i <= L.ni && j >= 0 && j < L.nj) {          // i-face (i, j)
        const double mx = 0.5 * (xn[j * W + i] + xn[(j + 1) * W + i]);
        const double my = 0.5 * (yn[j * W + i] + yn[(j + 1) * W + i]);
        const double dx = mx - px, dy = my - py;
        const double rx = px + (c * dx - s * dy), ry = py + (s * dx + c * dy);
        wix = -omega * (ry - py);
        wiy = omega * (rx - px);
    }
    if (i >= 0 && i < L.ni && j >= 0 && j <= L.nj) {          // j-face (i, j)
        const double mx = 0.5 * (xn[j * W + i] + xn[j * W + i + 1]);
        const double my = 0.5 * (yn[j * W + i] + yn[j * W + i + 1]);
        const double dx = mx - px, dy = my - py;
        const double rx = px + (c * dx - s * dy), ry = py + (s * dx + c * dy);
        wjx = -omega * (ry - py);
        wjy = omega * (rx - px);
    }
    geo[G_WIX * NS + t] = wix;
    geo[G_WIY * NS + t] = wiy;
    geo[G_WJX * NS + t] = wjx;
    geo[G_WJY * NS + t] = wjy;
}

// ghost cells: centre reflected across the boundary face (the partner's
// across the wake cut), volume and mean face vectors of the mirrored cell
__global__ void k_geom_ghost(Lay L, const double *xn, const double *yn, double *geo) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    int i, j;
    if (!decode(L, s, i, j) || interior(L, i, j)) return;
    const int NS = L.NS, W = L.ni + 1;
    auto X = [&](int I, int J) { return xn[J * W + I]; };
    auto Y = [&](int I, int J) { return yn[J * W + I]; };
    double cx, cy;
    int si, sj;
    g_centre<double>(L, X, Y, i, j, cx, cy, si, sj);
    const int msrc = L.slot(si, sj);
    geo[G_XC * NS + s] = cx;
    geo[G_YC * NS + s] = cy;
    geo[G_SB0 * NS + s] = geo[G_SB0 * NS + msrc];
    geo[G_SB1 * NS + s] = geo[G_SB1 * NS + msrc];
    geo[G_SB2 * NS + s] = geo[G_SB2 * NS + msrc];
    geo[G_SB3 * NS + s] = geo[G_SB3 * NS + msrc];
    geo[G_VOL * NS + s] = geo[G_VOL * NS + msrc];
}

// ---------------------------------------------------------- boundary states
// Section 2: no-slip walls and far-field conditions by Riemann invariants;
// two ghost layers, layer k from interior cell k; wake-cut ghosts are the
// partner cells.
__device__ void farfield(const double ui[4], const double uinf[4], double nx, double ny, double out[4]) {
    const double g1 = GAM - 1.0;
    double rho = ui[0];
    double vx = ui[1] / rho, vy = ui[2] / rho;
    double p = pres(ui[0], ui[1], ui[2], ui[3]);
    double a = sqrt(GAM * p / rho);
    double rinf = uinf[0];
    double vxf = uinf[1] / rinf, vyf = uinf[2] / rinf;
    double pf = pres(uinf[0], uinf[1], uinf[2], uinf[3]);
    double af = sqrt(GAM * pf / rinf);
    double vn = vx * nx + vy * ny;
    double vnf = vxf * nx + vyf * ny;
    double rp = vn + 2.0 * a / g1;
    double rm = vnf - 2.0 * af / g1;
    double vnb = 0.5 * (rp + rm);
    double ab = 0.25 * g1 * (rp - rm);
    bool outf = vnb > 0.0;
    double sent = outf ? p / pow(rho, GAM) : pf / pow(rinf, GAM);
    double tx = outf ? vx - vn * nx : vxf - vnf * nx;
    double ty = outf ? vy - vn * ny : vyf - vnf * ny;
    double base = ab * ab / (GAM * sent);
    double rhob = base * base * sqrt(base);
    double pb = rhob * ab * ab / GAM;
    double ub = tx + vnb * nx, vb = ty + vnb * ny;
    out[0] = rhob;
    out[1] = rhob * ub;
    out[2] = rhob * vb;
    out[3] = pb / g1 + 0.5 * rhob * (ub * ub + vb * vb);
}

__device__ inline void unit(double sx, double sy, double &nx, double &ny) {
    double ln = sqrt(sx * sx + sy * sy);
    nx = sx / ln;
    ny = sy / ln;
}

// a state seen from a boundary moving at (wx, wy) (sign +1: relative,
// -1: back to absolute): velocity shifted, density and pressure kept
__device__ void shift_frame(const double in[4], double wx, double wy, double sign, double out[4]) {
    const double rho = in[0];
    const double p = pres(in[0], in[1], in[2], in[3]);
    const double mx = in[1] - sign * (rho * wx), my = in[2] - sign * (rho * wy);
    out[0] = rho;
    out[1] = mx;
    out[2] = my;
    out[3] = p / (GAM - 1.0) + 0.5 * (mx * mx + my * my) / rho;
}

// far field of a boundary face moving at w (Riemann invariants of the
// velocity relative to the face)
__device__ void farfield_moving(const double ui[4], const double uinf[4], double nx, double ny, double wx,
                                double wy, double out[4]) {
    double ur[4], fr[4], br[4];
    shift_frame(ui, wx, wy, 1.0, ur);
    shift_frame(uinf, wx, wy, 1.0, fr);
    farfield(ur, fr, nx, ny, br);
    shift_frame(br, wx, wy, -1.0, out);
}

// ghost of a wall moving at w: no-slip v_g = 2 w - v, slip the relative
// velocity mirrored; density and pressure mirrored
__device__ void moving_wall(const double ui[4], double nx, double ny, double wx, double wy, int noslip,
                            double out[4]) {
    const double rho = ui[0];
    const double p = pres(ui[0], ui[1], ui[2], ui[3]);
    double mx, my;
    if (noslip) {
        mx = 2.0 * rho * wx - ui[1];
        my = 2.0 * rho * wy - ui[2];
    } else {
        const double rx = ui[1] - rho * wx, ry = ui[2] - rho * wy;
        const double rn = rx * nx + ry * ny;
        mx = (rx - 2.0 * rn * nx) + rho * wx;
        my = (ry - 2.0 * rn * ny) + rho * wy;
    }
    out[0] = rho;
    out[1] = mx;
    out[2] = my;
    out[3] = p / (GAM - 1.0) + 0.5 * (mx * mx + my * my) / rho;
}

// state of cell (i, j), i interior, j in [-2, nj+2)
__device__ void jrow_state(const Lay &L, const double *geo, const double *u, const Phys &ph,
                           int noslip, int i, int j, double out[4]) {
    const int NS = L.NS;
    if (j >= 0 && j < L.nj) {
        ld4(u, NS, L.slot(i, j), out);
        return;
    }
    if (j < 0) {
        int k = -1 - j;
        if (cut_col(L, i)) {
            ld4(u, NS, L.slot(L.ni - 1 - i, k), out);
            return;
        }
        double ui[4];
        ld4(u, NS, L.slot(i, k), ui);
        if (ph.ale) {
            int f = L.slot(i, 0);
            double nx, ny;
            unit(geo[G_SETA_X * NS + f], geo[G_SETA_Y * NS + f], nx, ny);
            moving_wall(ui, nx, ny, geo[G_WJX * NS + f], geo[G_WJY * NS + f], noslip, out);
        } else if (noslip) {
            out[0] = ui[0];
            out[1] = -ui[1];
            out[2] = -ui[2];
            out[3] = ui[3];
        } else {
            int f = L.slot(i, 0);
            double nx, ny;
            unit(geo[G_SETA_X * NS + f], geo[G_SETA_Y * NS + f], nx, ny);
            double mn = ui[1] * nx + ui[2] * ny;
            out[0] = ui[0];
            out[1] = ui[1] - 2.0 * mn * nx;
            out[2] = ui[2] - 2.0 * mn * ny;
            out[3] = ui[3];
        }
        return;
    }
    int k = j - L.nj;
    double ui[4];
    ld4(u, NS, L.slot(i, L.nj - 1 - k), ui);
    int f = L.slot(i, L.nj);
    double nx, ny;
    unit(geo[G_SETA_X * NS + f], geo[G_SETA_Y * NS + f], nx, ny);
    if (ph.ale) farfield_moving(ui, ph.uinf, nx, ny, geo[G_WJX * NS + f], geo[G_WJY * NS + f], out);
    else farfield(ui, ph.uinf, nx, ny, out);
}

// state of ghost cell (i, j) from the interior states (ghost states never
// read other ghosts, so all of them can be filled at once)
__device__ inline void ghost_state(const Lay &L, const double *geo, const double *u, const Phys &ph, int noslip,
                                   int i, int j, double out[4]) {
    const int NS = L.NS;
    if (i >= 0 && i < L.ni) {
        jrow_state(L, geo, u, ph, noslip, i, j, out);
        return;
    }
    int jc = min(max(j, 0), L.nj - 1);
    double src[4], nx, ny;
    int f;
    if (i < 0) {
        jrow_state(L, geo, u, ph, noslip, -1 - i, j, src);
        f = L.slot(0, jc);
        unit(-geo[G_SXI_X * NS + f], -geo[G_SXI_Y * NS + f], nx, ny);
    } else {
        jrow_state(L, geo, u, ph, noslip, L.ni - 1 - (i - L.ni), j, src);
        f = L.slot(L.ni, jc);
        unit(geo[G_SXI_X * NS + f], geo[G_SXI_Y * NS + f], nx, ny);
    }
    if (ph.ale) farfield_moving(src, ph.uinf, nx, ny, geo[G_WIX * NS + f], geo[G_WIY * NS + f], out);
    else farfield(src, ph.uinf, nx, ny, out);
}

// eddy viscosity ghosts: zero at walls, copy at far field, partner at the cut
__device__ double jrow_mut(const Lay &L, const double *mut, int i, int j) {
    if (j >= 0 && j < L.nj) return mut[L.slot(i, j)];
    if (j < 0) {
        int k = -1 - j;
        if (cut_col(L, i)) return mut[L.slot(L.ni - 1 - i, k)];
        return 0.0;
    }
    return mut[L.slot(i, L.nj - 1 - (j - L.nj))];
}

__global__ void k_mut_ghosts(BK b) {
    const BlockXY cb = xcd_block();
    LevelDev d;
    if (!take(b, cb.y, d)) return;
    const Lay L = d.L;
    double *mut = d.mut;
    int s = cb.x * blockDim.x + threadIdx.x;
    int i, j;
    if (!decode(L, s, i, j) || interior(L, i, j)) return;
    double v;
    if (i >= 0 && i < L.ni) v = jrow_mut(L, mut, i, j);
    else if (i < 0) v = jrow_mut(L, mut, -1 - i, j);
    else v = jrow_mut(L, mut, L.ni - 1 - (i - L.ni), j);
    mut[s] = v;
}

// ------------------------------------------------------- per-cell quantities
// Section 2: p, sensor quantity (entropy p/rho^gamma for RANS, pressure for
// Euler), spectral radii r = |v.S| + a|S| and the multidimensional
// correction of eq. "spectralcorrection"; temperature T = p / rho.
// normal velocities through the mean i- and j-faces, relative to a moving
// mesh (grid velocity omega x (r - pivot) at the cell centre)
__device__ inline void rel_normal(const Phys &ph, const double *geo, int NS, int s, double vx, double vy,
                                  double sb0, double sb1, double sb2, double sb3, double &vnx, double &vne) {
    vnx = vx * sb0 + vy * sb1;
    vne = vx * sb2 + vy * sb3;
    if (ph.ale) {
        const double wx = -ph.omega * (geo[G_YC * NS + s] - ph.py);
        const double wy = ph.omega * (geo[G_XC * NS + s] - ph.px);
        vnx = vnx - (wx * sb0 + wy * sb1);
        vne = vne - (wx * sb2 + wy * sb3);
    }
}

__device__ inline void cell_quantities(const Phys &ph, const double *geo, int NS, int s, int rans, const double U[4],
                                       double *cq) {
    double r = U[0], mx = U[1], my = U[2], E = U[3];
    double vx = mx / r, vy = my / r;
    double p = pres(r, mx, my, E);
    double a = sqrt(GAM * p / r);
    double q = rans ? p / pow(r, GAM) : p;
    double sb0 = geo[G_SB0 * NS + s], sb1 = geo[G_SB1 * NS + s];
    double sb2 = geo[G_SB2 * NS + s], sb3 = geo[G_SB3 * NS + s];
    double vnx, vne;
    rel_normal(ph, geo, NS, s, vx, vy, sb0, sb1, sb2, sb3, vnx, vne);
    double rxi = fabs(vnx) + a * sqrt(sb0 * sb0 + sb1 * sb1);
    double reta = fabs(vne) + a * sqrt(sb2 * sb2 + sb3 * sb3);
    double t = reta / rxi;
    double rtxi = rxi * (1.0 + cbrt(t * t));
    t = rxi / reta;
    double rteta = reta * (1.0 + cbrt(t * t));
    cq[Q_P * NS + s] = p;
    cq[Q_Q * NS + s] = q;
    cq[Q_RXI * NS + s] = rtxi;
    cq[Q_RETA * NS + s] = rteta;
    cq[Q_T * NS + s] = p / r;
}

// ghost states and cell quantities in one pass: a ghost cell's quantities
// need only its own (just computed) state
__global__ void k_ghost_cq(BK b, int noslip, int rans) {
    const BlockXY cb = xcd_block();
    LevelDev d;
    if (!take(b, cb.y, d)) return;
    const Lay L = d.L;
    const Phys ph = b.PH[cb.y];
    int s, i, j;   // every padded cell, -NG <= i < ni + NG, -NG <= j < nj + NG
    if (!rect_cell(L, cb.x * blockDim.x + threadIdx.x, L.NI, L.NJ, NG, s, i, j)) return;
    const int NS = L.NS;
    double U[4];
    if (interior(L, i, j)) {
#pragma unroll
        for (int k = 0; k < 4; ++k) U[k] = d.u[k * NS + s];
    } else {
        ghost_state(L, d.geo, d.u, ph, noslip, i, j, U);
#pragma unroll
        for (int k = 0; k < 4; ++k) d.u[k * NS + s] = U[k];
    }
    cell_quantities(ph, d.geo, NS, s, rans, U, d.cq);
}

// c* of the current cycle: the start-up value for n_ramp cycles, then
// geometric growth per cycle up to the target (Section 6 start-up)
__device__ inline double cfl_of(const Phys &ph, int n) {
    if (n < ph.n_ramp) return fmin(ph.cfl, ph.cfl_ramp);
    if (ph.ramp_growth > 1.0)
        return fmin(ph.cfl, ph.cfl_ramp * pow(ph.ramp_growth, (double)(n - ph.n_ramp + 1)));
    return ph.cfl;
}

// Section 4.1, dt* = c* times the local mesh width (reading): c* Omega /
// (r_xi + r_eta), or with dt_form 1 c* Omega / max(r_xi, r_eta), the
// smaller of the two directional CFL steps, of interior cell s
__device__ inline double local_dt(const Phys &ph, double cfl, const double *geo, const double *u, int NS, int s) {
    double r = u[s], mx = u[NS + s], my = u[2 * NS + s], E = u[3 * NS + s];
    double vx = mx / r, vy = my / r;
    double p = pres(r, mx, my, E);
    double a = sqrt(GAM * p / r);
    double sb0 = geo[G_SB0 * NS + s], sb1 = geo[G_SB1 * NS + s];
    double sb2 = geo[G_SB2 * NS + s], sb3 = geo[G_SB3 * NS + s];
    double vnx, vne;
    rel_normal(ph, geo, NS, s, vx, vy, sb0, sb1, sb2, sb3, vnx, vne);
    double rxi = fabs(vnx) + a * sqrt(sb0 * sb0 + sb1 * sb1);
    double reta = fabs(vne) + a * sqrt(sb2 * sb2 + sb3 * sb3);
    return cfl * geo[G_VOL * NS + s] / (ph.dt_form ? fmax(rxi, reta) : rxi + reta);
}

// Section 2: velocity and temperature gradients at vertices, Green-Gauss
// over the quadrilateral of the four surrounding cell centres.
__global__ void k_vertex_gradients(BK b) {
    const BlockXY cb = xcd_block();
    LevelDev d;
    if (!take(b, cb.y, d)) return;
    const Lay L = d.L;
    const double *geo = d.geo, *u = d.u, *cq = d.cq;
    double *vg = d.vg;
    int s, i, j;   // every vertex, 0 <= i <= ni, 0 <= j <= nj
    if (!rect_cell(L, cb.x * blockDim.x + threadIdx.x, L.ni + 1, L.nj + 1, 0, s, i, j)) return;
    const int NS = L.NS, NJ = L.NJ;
    const int c[4] = {s - (2 * NJ + 1), s - (NJ + 1), s, s - NJ};   // SW, SE, NE, NW
    double X[4], Y[4], U[4], V[4], T[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        X[k] = geo[G_XC * NS + c[k]];
        Y[k] = geo[G_YC * NS + c[k]];
        double r = u[c[k]];
        U[k] = u[NS + c[k]] / r;
        V[k] = u[2 * NS + c[k]] / r;
        T[k] = cq[Q_T * NS + c[k]];
    }
    double A = 0.5 * ((X[2] - X[0]) * (Y[3] - Y[1]) - (Y[2] - Y[0]) * (X[3] - X[1]));
    double g[6] = {0, 0, 0, 0, 0, 0};
    const double *phi[3] = {U, V, T};
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        double gx = 0.0, gy = 0.0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int a = e, b = (e + 1) & 3;
            double m = 0.5 * (phi[f][a] + phi[f][b]);
            double tx = m * (Y[b] - Y[a]);
            double ty = m * (X[a] - X[b]);
            if (e == 0) { gx = tx; gy = ty; }
            else { gx = gx + tx; gy = gy + ty; }
        }
        g[2 * f] = gx / A;
        g[2 * f + 1] = gy / A;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) vg[k * NS + s] = g[k];
}

// Baldwin-Lomax algebraic eddy viscosity (Section 2), j-cells walked from
// the wall / wake cut outward.  Ties in the maximum of F and the first
// inner/outer crossover go to the lowest j; the search is limited to the
// inner half of the column.
//
// A workgroup takes eight adjacent i-columns, 32 lanes each, lane l holding
// rows l, l + 32, ... of its column in registers.  In the skewed layout a
// cache line holds one cell of each of eight adjacent columns
// (slot(i - 1, j + 1) = slot(i, j) + 1), so one load instruction of the
// workgroup reads the same rows of eight adjacent columns from about 32
// cache lines instead of 256.  The column searches are 32-lane reductions,
// exact whatever their order (first j of the largest F, largest and
// smallest speed, first crossover j), and every per-cell expression is the
// scan's, so the eddy viscosity is that of a serial walk up the column.
// Groups of eight columns go to the XCDs in contiguous ranges.
constexpr int BL_TPB = 256, BL_COLS = 8, BL_LANES = 32;
constexpr int BL_MAXK = 16;                 // rows per lane: nj <= 512

// the scan's maximum of F: a NaN at the wall wins (a scan starting there
// never moves on), other NaNs never win, otherwise the larger F and then the
// smaller j; y is carried along with its row
struct BlMax {
    double f, y;
    int j;
};
__device__ inline BlMax bl_better(BlMax a, BlMax b) {
    const bool bn = b.f != b.f, an = a.f != a.f;
    bool take;
    if (bn || an) take = (bn && b.j == 0) || (!(an && a.j == 0) && !bn);
    else take = b.f > a.f || (b.f == a.f && b.j < a.j);
    return take ? b : a;
}

__global__ __launch_bounds__(BL_TPB) void k_baldwin_lomax(BK b) {
    LevelDev d;
    if (!take(b, blockIdx.y, d)) return;
    const Lay L = d.L;
    const int gx = gridDim.x;
    const int bx = xcd_range((int)blockIdx.x, gx);
    const int lane = threadIdx.x % BL_LANES;
    const int i = bx * BL_COLS + (int)threadIdx.x / BL_LANES;
    if (i >= L.ni) return;                  // a whole 32-lane group: its reductions stay inside it
    const double *geo = d.geo, *u = d.u, *cq = d.cq, *vg = d.vg;
    double *mut = d.mut;
    const Phys ph = b.PH[blockIdx.y];
    const int nj = L.nj, NS = L.NS, NJ = L.NJ;
    const bool cut = cut_col(L, i);
    auto omega = [&](int jj) {
        int s = L.slot(i, jj);
        int v0 = s, v1 = s + NJ, v2 = s + 2 * NJ + 1, v3 = s + NJ + 1;   // (i,j),(i+1,j),(i+1,j+1),(i,j+1)
        double w0 = vg[V_VX * NS + v0] - vg[V_UY * NS + v0];
        double w1 = vg[V_VX * NS + v1] - vg[V_UY * NS + v1];
        double w2 = vg[V_VX * NS + v2] - vg[V_UY * NS + v2];
        double w3 = vg[V_VX * NS + v3] - vg[V_UY * NS + v3];
        return fabs(0.25 * (((w0 + w1) + w2) + w3));
    };
    const int s0 = L.slot(i, 0);
    const double muw = sutherland(cq[Q_T * NS + s0], ph.mu_inf);
    const double rhow = u[s0];
    const double tauw = muw * omega(0);
    const double sq = sqrt(rhow * tauw);
    const int jb = nj / 2, jlim = jb > 1 ? jb : 1;      // the scan starts at the wall cell
    double yv[BL_MAXK], miv[BL_MAXK], rv[BL_MAXK];
    BlMax m = {-INFINITY, 0.0, nj};
    double smax = -INFINITY, smin = INFINITY;
#pragma unroll
    for (int k = 0; k < BL_MAXK; ++k) {
        const int jj = lane + BL_LANES * k;
        yv[k] = miv[k] = rv[k] = 0.0;
        if (jj < nj) {
            int s = L.slot(i, jj);
            double r = u[s];
            double vx = u[NS + s] / r, vy = u[2 * NS + s] / r;
            double om = omega(jj);
            double y = geo[G_WD * NS + s];
            double damp = 1.0;
            if (!cut) {
                double yplus = y * sq / muw;
                damp = 1.0 - exp(-yplus / BL_APLUS);
            }
            const double F = y * om * damp;
            const double sp = sqrt(vx * vx + vy * vy);
            double l = BL_KAPPA * y * damp;
            yv[k] = y;
            miv[k] = r * (l * l) * om;
            rv[k] = r;
            if (jj < jlim) {
                m = bl_better(m, BlMax{F, y, jj});
                smax = fmax(smax, sp);
                smin = fmin(smin, sp);
            }
        }
    }
#pragma unroll
    for (int o = BL_LANES / 2; o > 0; o >>= 1) {
        BlMax w;
        w.f = __shfl_xor(m.f, o);
        w.y = __shfl_xor(m.y, o);
        w.j = __shfl_xor(m.j, o);
        m = bl_better(m, w);
        smax = fmax(smax, __shfl_xor(smax, o));
        smin = fmin(smin, __shfl_xor(smin, o));
    }
    const double fm = m.f, ymax = m.y, udif = smax - smin;
    const double fwake = fm > 0.0 ? fmin(ymax * fm, BL_CWK * ymax * udif * udif / fm) : 0.0;
    auto outer = [&](int k) {
        double t = BL_CKLEB * yv[k] / ymax;
        double t2 = t * t;
        double fk = 1.0 / (1.0 + 5.5 * (t2 * t2 * t2));
        return rv[k] * BL_K * BL_CCP * fwake * fk;
    };
    int jc = jb;
#pragma unroll
    for (int k = 0; k < BL_MAXK; ++k) {
        const int jj = lane + BL_LANES * k;
        if (jj < jb && miv[k] >= outer(k)) jc = min(jc, jj);
    }
#pragma unroll
    for (int o = BL_LANES / 2; o > 0; o >>= 1) jc = min(jc, __shfl_xor(jc, o));
#pragma unroll
    for (int k = 0; k < BL_MAXK; ++k) {
        const int jj = lane + BL_LANES * k;
        if (jj < nj) mut[L.slot(i, jj)] = jj < jc ? miv[k] : outer(k);
    }
}

// -------------------------------------------------------------- residual
// JST face flux (Section 2) split into the central part (f^c) and the
// artificial dissipation / viscous part (f^v) of eq. "split-rhs".
struct FaceOut {
    double C[4], V[4];
};

__device__ void face_flux(const Lay &L, const double *geo, const double *u, const double *cq,
                          const double *vg, const double *mut, const Phys &ph, const ResArgs &a,
                          int sL, int sR, int off, double sx, double sy, int gL, int gR, bool wall,
                          int sf, int wplane, FaceOut &o) {
    const int NS = L.NS;
    double UL[4], UR[4];
    ld4(u, NS, sL, UL);
    ld4(u, NS, sR, UR);
    double pL = cq[Q_P * NS + sL], pR = cq[Q_P * NS + sR];
    // moving mesh: grid flux w . S of the face (grid velocity at its midpoint)
    const double q = ph.ale ? geo[wplane * NS + sf] * sx + geo[(wplane + 1) * NS + sf] * sy : 0.0;
    if (wall) {
        double pw = 0.5 * (pL + pR);
        o.C[0] = 0.0;
        o.C[1] = pw * sx;
        o.C[2] = pw * sy;
        o.C[3] = ph.ale ? pw * q : 0.0;     // pressure work of a moving wall
#pragma unroll
        for (int k = 0; k < 4; ++k) o.V[k] = 0.0;
    } else {
        double qsL = UL[1] * sx + UL[2] * sy, vsL = qsL / UL[0];
        double qsR = UR[1] * sx + UR[2] * sy, vsR = qsR / UR[0];
        double FL[4] = {qsL, UL[1] * vsL + pL * sx, UL[2] * vsL + pL * sy, (UL[3] + pL) * vsL};
        double FR[4] = {qsR, UR[1] * vsR + pR * sx, UR[2] * vsR + pR * sy, (UR[3] + pR) * vsR};
#pragma unroll
        for (int k = 0; k < 4; ++k) o.C[k] = 0.5 * (FL[k] + FR[k]);
        if (ph.ale) {
#pragma unroll
            for (int k = 0; k < 4; ++k) o.C[k] = o.C[k] - q * (0.5 * (UL[k] + UR[k]));
        }
        const int rp = (off == L.NJ ? Q_RXI : Q_RETA) * NS;
        double rf = fmax(cq[rp + sL], cq[rp + sR]);
        double wL[4] = {UL[0], UL[1], UL[2], UL[3] + pL};
        double wR[4] = {UR[0], UR[1], UR[2], UR[3] + pR};
        double d[4];
        if (a.fine) {
            const double *q = cq + Q_Q * NS;
            double qLL = q[sL - off], qL = q[sL], qR = q[sR], qRR = q[sR + off];
            double sLs = fabs(((qR - 2.0 * qL) + qLL) / (((qR + 2.0 * qL) + qLL) + 0.001));
            double sRs = fabs(((qRR - 2.0 * qR) + qL) / (((qRR + 2.0 * qR) + qL) + 0.001));
            double sf = fmin(0.25, fmax(sLs, sRs));
            double e2 = sf * rf;
            double e4 = fmax(0.0, rf / 32.0 - 2.0 * e2);
            double ULL[4], URR[4];
            ld4(u, NS, sL - off, ULL);
            ld4(u, NS, sR + off, URR);
            double pLL = cq[Q_P * NS + sL - off], pRR = cq[Q_P * NS + sR + off];
            double wLL[4] = {ULL[0], ULL[1], ULL[2], ULL[3] + pLL};
            double wRR[4] = {URR[0], URR[1], URR[2], URR[3] + pRR};
#pragma unroll
            for (int k = 0; k < 4; ++k)
                d[k] = e2 * (wR[k] - wL[k]) - e4 * (((wRR[k] - 3.0 * wR[k]) + 3.0 * wL[k]) - wLL[k]);
        } else {
            double e2 = ph.kappa2c * rf;
#pragma unroll
            for (int k = 0; k < 4; ++k) d[k] = e2 * (wR[k] - wL[k]);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) o.V[k] = -d[k];
    }
    if (a.viscous) {
        // Section 2: face gradient = mean of the two end-vertex gradients
        double fux = 0.5 * (vg[V_UX * NS + gL] + vg[V_UX * NS + gR]);
        double fuy = 0.5 * (vg[V_UY * NS + gL] + vg[V_UY * NS + gR]);
        double fwx = 0.5 * (vg[V_VX * NS + gL] + vg[V_VX * NS + gR]);
        double fwy = 0.5 * (vg[V_VY * NS + gL] + vg[V_VY * NS + gR]);
        double fTx = 0.5 * (vg[V_TX * NS + gL] + vg[V_TX * NS + gR]);
        double fTy = 0.5 * (vg[V_TY * NS + gL] + vg[V_TY * NS + gR]);
        double fvx = 0.5 * (UL[1] / UL[0] + UR[1] / UR[0]);
        double fvy = 0.5 * (UL[2] / UL[0] + UR[2] / UR[0]);
        double fT = 0.5 * (cq[Q_T * NS + sL] + cq[Q_T * NS + sR]);
        double mu = sutherland(fT, ph.mu_inf);
        double mt = 0.5 * (mut[sL] + mut[sR]);
        double mue = mu + mt;
        double kc = (mu / ph.pr + mt / ph.prt) * (GAM / (GAM - 1.0));
        double div = fux + fwy;
        double txx = mue * (2.0 * fux - (2.0 / 3.0) * div);
        double tyy = mue * (2.0 * fwy - (2.0 / 3.0) * div);
        double txy = mue * (fuy + fwx);
        double qx = kc * fTx, qy = kc * fTy;
        double G1 = txx * sx + txy * sy;
        double G2 = txy * sx + tyy * sy;
        double G3 = ((fvx * txx + fvy * txy) + qx) * sx + ((fvx * txy + fvy * tyy) + qy) * sy;
        o.V[1] = o.V[1] - G1;
        o.V[2] = o.V[2] - G2;
        o.V[3] = o.V[3] - G3;
    }
}

// The cell's part of the residual once its face sums are known (Section 2
// and eq. "split-rhs"): BDF time derivative, FAS forcing, then either F, or
// the smoother stage's blended f^v accumulator and g = D^-1 (dt*) r.
template <typename BT>
__device__ inline void residual_cell(const LevelDev &d, const ResArgs &a, int NS, int s, double Fc[4],
                                     double Fv[4]) {
    const double *u = d.u, *un = d.un, *unm1 = d.unm1, *src = d.src, *dts = d.dts;
    double *F = d.F, *acc = d.acc;
    const BT *blk = (const BT *)d.blk;
    BT *g = (BT *)d.g;
    if (a.bdf) {
        double uu[4], u1[4];
        ld4(u, NS, s, uu);
        ld4(un, NS, s, u1);
        if (a.bdf == 2) {
            double u2[4];
            ld4(unm1, NS, s, u2);
#pragma unroll
            for (int k = 0; k < 4; ++k) Fc[k] = Fc[k] + ((3.0 * uu[k] - 4.0 * u1[k]) + u2[k]) / (2.0 * a.dt);
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) Fc[k] = Fc[k] + (uu[k] - u1[k]) / a.dt;
        }
    }
    if (a.forcing) {
#pragma unroll
        for (int k = 0; k < 4; ++k) Fc[k] = Fc[k] - src[k * NS + s];
    }
    if (a.mode == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double f = Fc[k] + Fv[k];
            F[k * NS + s] = f;
            if (a.src_acc) d.src[k * NS + s] = f + acc[k * NS + s];
        }
        return;
    }
    double r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double av = Fv[k];
        if (a.stage > 0) av = a.beta * Fv[k] + (1.0 - a.beta) * acc[k * NS + s];
        acc[k * NS + s] = av;
        r[k] = Fc[k] + av;
    }
    if (a.aw) {
        const double dt_s = dts[s];
#pragma unroll
        for (int k = 0; k < 4; ++k) r[k] = dt_s * r[k];
    }
    BT rb[4] = {(BT)r[0], (BT)r[1], (BT)r[2], (BT)r[3]};
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        BT acc4 = (BT)0;
#pragma unroll
        for (int c = 0; c < 4; ++c) acc4 = fma(blk[BL<BT>::at(B_DINV, NS, s, rr, c)], rb[c], acc4);
        g[rr * NS + s] = acc4;
    }
}

// Residual of a level (Section 2; eq. "split-rhs" for the stages): the face
// fluxes of each cell's four faces, summed as (e - w) + (n - s) per
// component and divided by the volume, then residual_cell.  A cell's west
// face is the face between cells i - 1 and i, formed by face_flux from the
// two cells' slots, the face vector stored at the cell and the two vertices
// of the face; its east face is the west face of cell i + 1, argument for
// argument, and likewise for the south and north faces.
//
// Large launches: one workgroup per tile of RT_I x RT_J cells, every face of
// the tile computed once.  The i-faces ((RT_I + 1) x RT_J, the west face of
// each cell and the east face of the tile's last column) and the j-faces
// (RT_I x (RT_J + 1)) are written to LDS plane by plane, and each cell then
// sums its four: the result is bitwise that of the four-lane kernel below,
// with half the flux evaluations of a per-cell kernel and neighbouring
// faces' gathers served by the same cache lines.
// (16 x 15 cells: 255 i-faces and 256 j-faces, so each of the 256 threads
// forms at most one face of each family)
constexpr int RT_I = 16, RT_J = 15, RT_TPB = 256;
constexpr int RT_NIF = (RT_I + 1) * RT_J, RT_NJF = RT_I * (RT_J + 1);

// Batches launch one row of workgroups over the tiles of all cases in turn
// (b.tile0: first tile of each case), so that the XCD runs of xcd_block
// hold real tiles only and split them evenly over the XCDs; one state
// launches its tiles (gridDim.x) for case blockIdx.y.
template <typename BT>
__global__ __launch_bounds__(RT_TPB) void k_residual_t(BK b, ResArgs a) {
    __shared__ double fi_c[4][RT_NIF], fi_v[4][RT_NIF], fj_c[4][RT_NJF], fj_v[4][RT_NJF];
    const BlockXY cb = xcd_block();
    int c = cb.y, tile = cb.x;
    if (b.tile0 != nullptr) {
        int lo = 0, hi = b.n;                           // b.tile0[lo] <= tile < b.tile0[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (b.tile0[mid] <= tile) lo = mid;
            else hi = mid;
        }
        c = lo;
        tile -= b.tile0[lo];
    }
    LevelDev d;
    if (!take(b, c, d)) return;
    const Lay L = d.L;
    const int nti = (L.ni + RT_I - 1) / RT_I, ntj = (L.nj + RT_J - 1) / RT_J;
    if (tile >= nti * ntj) return;                      // tile past this case's grid
    const Phys ph = b.PH[c];
    const int i0 = (tile % nti) * RT_I, j0 = (tile / nti) * RT_J;
    const int ci = min(RT_I, L.ni - i0), cj = min(RT_J, L.nj - j0);
    const int NS = L.NS, NJ = L.NJ, t = threadIdx.x;
    const double *geo = d.geo, *u = d.u, *cq = d.cq, *vg = d.vg, *mut = d.mut;
    // i-faces: face (fi, fj) is the west face of cell (i0 + fi, j0 + fj)
    static_assert(RT_NIF <= RT_TPB && RT_NJF <= RT_TPB, "one face of each family per thread");
    if (t < (ci + 1) * cj) {
        const int fi = t % (ci + 1), fj = t / (ci + 1);
        const int s = L.slot(i0 + fi, j0 + fj);
        FaceOut o;
        face_flux(L, geo, u, cq, vg, mut, ph, a, s - NJ, s, NJ, geo[G_SXI_X * NS + s], geo[G_SXI_Y * NS + s], s,
                  s + NJ + 1, false, s, G_WIX, o);
        const int q = fj * (RT_I + 1) + fi;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            fi_c[k][q] = o.C[k];
            fi_v[k][q] = o.V[k];
        }
    }
    // j-faces: face (fi, fj) is the south face of cell (i0 + fi, j0 + fj)
    if (t < ci * (cj + 1)) {
        const int fi = t % ci, fj = t / ci;
        const int i = i0 + fi, j = j0 + fj;
        const int s = L.slot(i, j);
        const bool wall = (j == 0) && !cut_col(L, i);
        FaceOut o;
        face_flux(L, geo, u, cq, vg, mut, ph, a, s - NJ - 1, s, NJ + 1, geo[G_SETA_X * NS + s],
                  geo[G_SETA_Y * NS + s], s, s + NJ, wall, s, G_WJX, o);
        const int q = fj * RT_I + fi;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            fj_c[k][q] = o.C[k];
            fj_v[k][q] = o.V[k];
        }
    }
    __syncthreads();
    const int ti = t % RT_I, tj = t / RT_I;
    if (ti >= ci || tj >= cj) return;
    const int s = L.slot(i0 + ti, j0 + tj);
    const int qw = tj * (RT_I + 1) + ti, qs = tj * RT_I + ti;
    const double vol = geo[G_VOL * NS + s];
    double Fc[4], Fv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double fc = (fi_c[k][qw + 1] - fi_c[k][qw]) + (fj_c[k][qs + RT_I] - fj_c[k][qs]);
        double fv = (fi_v[k][qw + 1] - fi_v[k][qw]) + (fj_v[k][qs + RT_I] - fj_v[k][qs]);
        Fc[k] = fc / vol;
        Fv[k] = fv / vol;
    }
    residual_cell<BT>(d, a, NS, s, Fc, Fv);
}

// Small launches: four lanes per cell, one face each (w, e, s, n), so the
// flux chain each lane runs is a quarter as long.  The face sums are formed
// by lane shuffles in the same order, (e - w) + (n - s), so the
// result is bitwise the same; lanes past the last cell redo cell 0 and store
// nothing, so every lane takes part in the shuffles.
template <typename BT>
__global__ __launch_bounds__(TPB) void k_residual_q(BK b, ResArgs a) {
    const BlockXY cb = xcd_block();
    LevelDev d;
    if (!take(b, cb.y, d)) return;
    const Lay L = d.L;
    const Phys ph = b.PH[cb.y];
    const int t = cb.x * blockDim.x + threadIdx.x;
    const int q = t & 3;
    int s, i, j;
    const bool valid = interior_cell(L, t >> 2, s, i, j);
    if (!valid) interior_cell(L, 0, s, i, j);
    const int NS = L.NS, NJ = L.NJ;
    // q = 0 west, 1 east (i-faces), 2 south, 3 north (j-faces); sf is the
    // face's slot (face vector, grid velocity) and also its first vertex
    const int sf = q == 0 ? s : q == 1 ? s + NJ : q == 2 ? s : s + NJ + 1;
    const int sL = q == 0 ? s - NJ : q == 2 ? s - NJ - 1 : s;
    const int sR = q == 0 ? s : q == 1 ? s + NJ : q == 2 ? s : s + NJ + 1;
    const int gR = q == 0 ? s + NJ + 1 : q == 2 ? s + NJ : s + 2 * NJ + 1;
    const int off = q < 2 ? NJ : NJ + 1;
    const int px = q < 2 ? G_SXI_X : G_SETA_X, py = q < 2 ? G_SXI_Y : G_SETA_Y;
    const bool wall = q == 2 && j == 0 && !cut_col(L, i);
    FaceOut o;
    face_flux(L, d.geo, d.u, d.cq, d.vg, d.mut, ph, a, sL, sR, off, d.geo[px * NS + sf], d.geo[py * NS + sf], sf,
              gR, wall, sf, q < 2 ? G_WIX : G_WJX, o);
    const double vol = d.geo[G_VOL * NS + s];
    double Fc[4], Fv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        // odd lanes: e - w and n - s (the partner is the even lane below)
        const double dc = o.C[k] - __shfl_xor(o.C[k], 1);
        const double dv = o.V[k] - __shfl_xor(o.V[k], 1);
        // lane 1: (e - w) + (n - s)
        const double fc = dc + __shfl_xor(dc, 2);
        const double fv = dv + __shfl_xor(dv, 2);
        Fc[k] = fc / vol;
        Fv[k] = fv / vol;
    }
    if (!valid || q != 1) return;
    residual_cell<BT>(d, a, NS, s, Fc, Fv);
}

// -------------------------------------------------- preconditioner blocks
// Section 4.4: A+- = (A +- |A|_c)/2 at the arithmetic mean of the two cell
// states, |A|_c = R |Lambda|_c R^-1 with the cutoff of eq. "cutoff"; here
// |A|_c = |l1| I + (|l3| - |l1|) r3 l3^T + (|l4| - |l1|) r4 l4^T (same
// matrix, the two acoustic projections written out).
__device__ void split_face(const double UL[4], const double UR[4], double sx, double sy, double d,
                           double qf, int ale, double Ap[16], double Am[16]) {
    double ln = sqrt(sx * sx + sy * sy);
    double nx = sx / ln, ny = sy / ln;
    double U0 = 0.5 * (UL[0] + UR[0]), U1 = 0.5 * (UL[1] + UR[1]);
    double U2 = 0.5 * (UL[2] + UR[2]), U3 = 0.5 * (UL[3] + UR[3]);
    double uu = U1 / U0, vv = U2 / U0;
    double p = pres(U0, U1, U2, U3);
    double a = sqrt(GAM * p / U0);
    double H = (U3 + p) / U0;
    const double g1 = GAM - 1.0;
    double q2 = uu * uu + vv * vv;
    double phi = 0.5 * g1 * q2;
    double V = uu * nx + vv * ny;
    double A[16] = {0.0, nx, ny, 0.0,
                    phi * nx - uu * V, V - (GAM - 2.0) * uu * nx, uu * ny - g1 * vv * nx, g1 * nx,
                    phi * ny - vv * V, vv * nx - g1 * uu * ny, V - (GAM - 2.0) * vv * ny, g1 * ny,
                    V * (phi - H), H * nx - g1 * uu * V, H * ny - g1 * vv * V, GAM * V};
    double lam[3] = {V, V + a, V - a};
    if (ale) {
        // moving face: F.n - w_n u, Jacobian and eigenvalues shifted by w_n
        const double sh = qf / ln;
#pragma unroll
        for (int k = 0; k < 4; ++k) A[k * 5] = A[k * 5] - sh;
        lam[0] = lam[0] - sh;
        lam[1] = lam[1] - sh;
        lam[2] = lam[2] - sh;
    }
    double al[3];
    double ad = a * d;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double m = fabs(lam[k]);
        al[k] = (d > 0.0 && m <= ad) ? 0.5 * (ad + m * m / ad) : m;
    }
    double b = g1 / (a * a);
    double r3[4] = {1.0, uu + a * nx, vv + a * ny, H + a * V};
    double r4[4] = {1.0, uu - a * nx, vv - a * ny, H - a * V};
    double l3[4] = {0.5 * (0.5 * b * q2 - V / a), 0.5 * (nx / a - b * uu), 0.5 * (ny / a - b * vv), 0.5 * b};
    double l4[4] = {0.5 * (0.5 * b * q2 + V / a), 0.5 * (-nx / a - b * uu), 0.5 * (-ny / a - b * vv), 0.5 * b};
    double c3 = al[1] - al[0], c4 = al[2] - al[0];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double absA = (r == c ? al[0] : 0.0) + c3 * r3[r] * l3[c] + c4 * r4[r] * l4[c];
            Ap[r * 4 + c] = ln * (0.5 * (A[r * 4 + c] + absA));
            Am[r * 4 + c] = ln * (0.5 * (A[r * 4 + c] - absA));
        }
    }
}

// scalar thin-layer estimate of the viscous flux Jacobian of a face
__device__ double visc_face(const Lay &L, const double *geo, const double *u, const double *cq,
                            const double *mut, const Phys &ph, int sL, int sR, double sx, double sy) {
    const int NS = L.NS;
    double rf = 0.5 * (u[sL] + u[sR]);
    double Tf = 0.5 * (cq[Q_T * NS + sL] + cq[Q_T * NS + sR]);
    double mue = sutherland(Tf, ph.mu_inf) + 0.5 * (mut[sL] + mut[sR]);
    double s2 = sx * sx + sy * sy;
    double vf = 0.5 * (geo[G_VOL * NS + sL] + geo[G_VOL * NS + sR]);
    return ((mue * (GAM / ph.pr)) * s2) / (rf * vf);
}

__device__ void face_blocks(const Lay &L, const double *geo, const double *u, const double *cq,
                            const double *mut, const Phys &ph, int viscous, int sL, int sR,
                            int plane_x, int plane_y, int sf, double Ap[16], double Am[16]) {
    const int NS = L.NS;
    double UL[4], UR[4];
    ld4(u, NS, sL, UL);
    ld4(u, NS, sR, UR);
    double sx = geo[plane_x * NS + sf], sy = geo[plane_y * NS + sf];
    double qf = 0.0;
    if (ph.ale) {
        const int wp = plane_x == G_SXI_X ? G_WIX : G_WJX;
        qf = geo[wp * NS + sf] * sx + geo[(wp + 1) * NS + sf] * sy;
    }
    split_face(UL, UR, sx, sy, ph.d_cut, qf, ph.ale, Ap, Am);
    if (viscous) {
        double v = visc_face(L, geo, u, cq, mut, ph, sL, sR, sx, sy);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            Ap[k * 5] = Ap[k * 5] + v;
            Am[k * 5] = Am[k * 5] - v;
        }
    }
}

// Row r of block b of cell s, written as wide stores: one 16-byte store in
// FP32 (the row is contiguous), two in FP64 (one per half plane).  A lane's
// stores go to its own cell's record, so a wave's store instruction touches
// one cache line per lane whatever the width: wider stores mean fewer of
// them.
template <typename BT> struct RowStore;
template <> struct RowStore<float> {
    __device__ static void put(float *blk, int b, int NS, int s, int r, const double (&v)[4]) {
        *reinterpret_cast<float4 *>(blk + BL<float>::at(b, NS, s, r, 0)) =
            make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
    }
};
template <> struct RowStore<double> {
    __device__ static void put(double *blk, int b, int NS, int s, int r, const double (&v)[4]) {
        *reinterpret_cast<double2 *>(blk + BL<double>::at(b, NS, s, r, 0)) = make_double2(v[0], v[1]);
        *reinterpret_cast<double2 *>(blk + BL<double>::at(b, NS, s, r, 2)) = make_double2(v[2], v[3]);
    }
};

// Block stores of k_blocks staged through the wave's LDS: every lane puts
// its cell's record of a plane (64 bytes) into LDS, then each store
// instruction writes 16 whole records, four lanes per record, so a cache
// line is written by one instruction instead of in four partial pieces.
// sc / vc: slot and validity of the cell whose record a lane writes in each
// of the four rounds (cells 16 k + lane / 4).
struct StageSlots {
    int sc[4], vc[4];
};
// FP64: two half planes per block (columns 0-1 and 2-3)
__device__ inline void block_out(double *blk, double *lds, const StageSlots &st, int b, int NS, int s,
                                 const double (&v)[16]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        double2 *mine = reinterpret_cast<double2 *>(lds + lane * 8);
#pragma unroll
        for (int r = 0; r < 4; ++r) mine[r] = make_double2(v[r * 4 + 2 * h], v[r * 4 + 2 * h + 1]);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int c = k * 16 + (lane >> 2), q = lane & 3;
            const double2 x = reinterpret_cast<const double2 *>(lds)[c * 4 + q];
            if (st.vc[k]) reinterpret_cast<double2 *>(blk + ((size_t)(2 * b + h) * NS + st.sc[k]) * 8)[q] = x;
        }
        __builtin_amdgcn_wave_barrier();
    }
}
// FP32: one plane per block, a cell's 16 values in 64 bytes
__device__ inline void block_out(float *blk, double *ldsd, const StageSlots &st, int b, int NS, int s,
                                 const double (&v)[16]) {
    const int lane = threadIdx.x & 63;
    float *lds = reinterpret_cast<float *>(ldsd);
    float4 *mine = reinterpret_cast<float4 *>(lds + lane * 16);
#pragma unroll
    for (int r = 0; r < 4; ++r)
        mine[r] = make_float4((float)v[r * 4], (float)v[r * 4 + 1], (float)v[r * 4 + 2], (float)v[r * 4 + 3]);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = k * 16 + (lane >> 2), q = lane & 3;
        const float4 x = reinterpret_cast<const float4 *>(lds)[c * 4 + q];
        if (st.vc[k]) reinterpret_cast<float4 *>(blk + ((size_t)b * NS + st.sc[k]) * 16)[q] = x;
    }
    __builtin_amdgcn_wave_barrier();
}

template <typename BT>
__global__ __launch_bounds__(TPB) void k_blocks(BK b, int aw, double tau, int viscous, int copy_u0) {
    const BlockXY cb = xcd_block();
    LevelDev dv;
    if (!take(b, cb.y, dv)) return;
    const Lay L = dv.L;
    const double *geo = dv.geo, *u = dv.u, *cq = dv.cq, *mut = dv.mut;
    BT *blk = (BT *)dv.blk;
    const Phys ph = b.PH[cb.y];
    int s, i, j;
    // lanes past the last cell form cell 0 again and write nothing: the
    // whole wave takes part in the staged block stores
    const bool valid = interior_cell(L, cb.x * blockDim.x + threadIdx.x, s, i, j);
    if (__builtin_amdgcn_ballot_w64(valid) == 0) return;
    if (!valid) interior_cell(L, 0, s, i, j);
    __shared__ __attribute__((aligned(16))) double lds[64 * 8];
    StageSlots stg;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = k * 16 + ((threadIdx.x & 63) >> 2);
        stg.sc[k] = __shfl(s, c);
        stg.vc[k] = __shfl((int)valid, c);
    }
    const int NS = L.NS, NJ = L.NJ;
    // the iteration's frozen dt* (read by the stages' residuals and sweeps)
    const double dt_s = local_dt(ph, cfl_of(ph, b.cyc[cb.y]), geo, u, NS, s);
    if (valid) dv.dts[s] = dt_s;
    if (copy_u0 && valid) {
#pragma unroll
        for (int k = 0; k < 4; ++k) dv.u0[k * NS + s] = u[k * NS + s];
    }
    double c, diag;
    if (aw) {
        double e = ph.eta * dt_s;
        c = e / geo[G_VOL * NS + s];
        diag = 1.0 + tau * e;
    } else {
        c = 1.0 / geo[G_VOL * NS + s];
        diag = tau;
    }
    // pass 1: D = c (((Xp_e - Xm_w) + Ep_n) - Em_s) + diag I; each face's
    // other block is kept for its off-diagonal slot (pass 2)
    double Ap[16], Am[16], acc[16], Bw[16], Be[16], Bs[16], Bn[16];
    face_blocks(L, geo, u, cq, mut, ph, viscous, s, s + NJ, G_SXI_X, G_SXI_Y, s + NJ, Ap, Am);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        acc[k] = Ap[k];
        Be[k] = Am[k];
    }
    face_blocks(L, geo, u, cq, mut, ph, viscous, s - NJ, s, G_SXI_X, G_SXI_Y, s, Ap, Am);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        acc[k] = acc[k] - Am[k];
        Bw[k] = Ap[k];
    }
    face_blocks(L, geo, u, cq, mut, ph, viscous, s, s + NJ + 1, G_SETA_X, G_SETA_Y, s + NJ + 1, Ap, Am);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        acc[k] = acc[k] + Ap[k];
        Bn[k] = Am[k];
    }
    face_blocks(L, geo, u, cq, mut, ph, viscous, s - NJ - 1, s, G_SETA_X, G_SETA_Y, s, Ap, Am);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        acc[k] = acc[k] - Am[k];
        Bs[k] = Ap[k];
    }
    double D[16], Di[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        D[k] = c * acc[k];
        Di[k] = (k % 5 == 0) ? 1.0 : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) D[k * 5] = D[k * 5] + diag;
    // Gauss-Jordan inverse without pivoting
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double piv = 1.0 / D[k * 5];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            D[k * 4 + cc] *= piv;
            Di[k * 4 + cc] *= piv;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (r == k) continue;
            double f = D[r * 4 + k];
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
                D[r * 4 + cc] = fma(-f, D[k * 4 + cc], D[r * 4 + cc]);
                Di[r * 4 + cc] = fma(-f, Di[k * 4 + cc], Di[r * 4 + cc]);
            }
        }
    }
    block_out(blk, lds, stg, B_DINV, NS, s, Di);
    // pass 2: M_slot = D^-1 B_slot
    const bool has[4] = {i > 0, i < L.ni - 1, j > 0 || cut_col(L, i), j < L.nj - 1};
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) {
        double B[16];
        if (has[sl]) {
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                if (sl == 0) B[k] = -(c * Bw[k]);
                else if (sl == 1) B[k] = c * Be[k];
                else if (sl == 2) B[k] = -(c * Bs[k]);
                else B[k] = c * Bn[k];
            }
        }
        double M[16];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
                double m = 0.0;
                if (has[sl]) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) m = fma(Di[r * 4 + k], B[k * 4 + cc], m);
                }
                M[r * 4 + cc] = m;
            }
        }
        block_out(blk, lds, stg, B_M0 + sl, NS, s, M);
    }
}

// Small launches: four lanes per cell, one face each, in k_blocks's face
// order (q = 0 east, 1 west, 2 north, 3 south).  Every lane gathers the four
// faces' diagonal contributions by shuffles and forms D = c (((X_e - X_w) +
// X_n) - X_s) + diag I and its inverse exactly as k_blocks does; lane q then
// writes row q of D^-1 and its own face's off-diagonal block D^-1 B.  The
// arithmetic is k_blocks's, so the blocks are bitwise the same; lanes past
// the last cell redo cell 0 and store nothing.
template <typename BT>
__global__ __launch_bounds__(TPB) void k_blocks_q(BK b, int aw, double tau, int viscous, int copy_u0) {
    const BlockXY cb = xcd_block();
    LevelDev dv;
    if (!take(b, cb.y, dv)) return;
    const Lay L = dv.L;
    const double *geo = dv.geo, *u = dv.u, *cq = dv.cq, *mut = dv.mut;
    BT *blk = (BT *)dv.blk;
    const Phys ph = b.PH[cb.y];
    const int t = cb.x * blockDim.x + threadIdx.x;
    const int q = t & 3;
    int s, i, j;
    const bool valid = interior_cell(L, t >> 2, s, i, j);
    if (!valid) interior_cell(L, 0, s, i, j);
    const int NS = L.NS, NJ = L.NJ;
    const double dt_s = local_dt(ph, cfl_of(ph, b.cyc[cb.y]), geo, u, NS, s);
    if (valid && q == 0) {
        dv.dts[s] = dt_s;
        if (copy_u0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) dv.u0[k * NS + s] = u[k * NS + s];
        }
    }
    double c, diag;
    if (aw) {
        double e = ph.eta * dt_s;
        c = e / geo[G_VOL * NS + s];
        diag = 1.0 + tau * e;
    } else {
        c = 1.0 / geo[G_VOL * NS + s];
        diag = tau;
    }
    const int sL = q == 0 ? s : q == 1 ? s - NJ : q == 2 ? s : s - NJ - 1;
    const int sR = q == 0 ? s + NJ : q == 1 ? s : q == 2 ? s + NJ + 1 : s;
    const int sf = q == 0 ? s + NJ : q == 1 ? s : q == 2 ? s + NJ + 1 : s;
    double Ap[16], Am[16];
    face_blocks(L, geo, u, cq, mut, ph, viscous, sL, sR, q < 2 ? G_SXI_X : G_SETA_X, q < 2 ? G_SXI_Y : G_SETA_Y, sf,
                Ap, Am);
    // this face's part of D (X) and its off-diagonal block (Bf)
    const bool plus = (q & 1) == 0;   // east and north add A+, west and south subtract A-
    double X[16], Bf[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        X[k] = plus ? Ap[k] : Am[k];
        Bf[k] = plus ? Am[k] : Ap[k];
    }
    double D[16], Di[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const double xe = __shfl(X[k], 0, 4), xw = __shfl(X[k], 1, 4);
        const double xn = __shfl(X[k], 2, 4), xs = __shfl(X[k], 3, 4);
        const double acc = ((xe - xw) + xn) - xs;
        D[k] = c * acc;
        Di[k] = (k % 5 == 0) ? 1.0 : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) D[k * 5] = D[k * 5] + diag;
    // Gauss-Jordan inverse without pivoting
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double piv = 1.0 / D[k * 5];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            D[k * 4 + cc] *= piv;
            Di[k * 4 + cc] *= piv;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (r == k) continue;
            double f = D[r * 4 + k];
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
                D[r * 4 + cc] = fma(-f, D[k * 4 + cc], D[r * 4 + cc]);
                Di[r * 4 + cc] = fma(-f, Di[k * 4 + cc], Di[r * 4 + cc]);
            }
        }
    }
    if (!valid) return;
    {
        double row[4];
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if ((k >> 2) == q) row[k & 3] = Di[k];
        RowStore<BT>::put(blk, B_DINV, NS, s, q, row);
    }
    // M_slot = D^-1 B_slot for this lane's face: slot 1 east, 0 west, 3 north,
    // 2 south; the west and south blocks enter with a minus sign
    const int sl = q == 0 ? 1 : q == 1 ? 0 : q == 2 ? 3 : 2;
    const bool has = sl == 0 ? i > 0 : sl == 1 ? i < L.ni - 1 : sl == 2 ? (j > 0 || cut_col(L, i)) : j < L.nj - 1;
    double B[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) B[k] = plus ? c * Bf[k] : -(c * Bf[k]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        double row[4];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            double m = 0.0;
            if (has) {
#pragma unroll
                for (int k = 0; k < 4; ++k) m = fma(Di[r * 4 + k], B[k * 4 + cc], m);
            }
            row[cc] = m;
        }
        RowStore<BT>::put(blk, B_M0 + sl, NS, s, r, row);
    }
}

// ------------------------------------------------------------- SGS sweeps
// Eq. "sgs-precon": x = P^-1 r, P = (D+L) D^-1 (D+U), by a forward and a
// backward block Gauss-Seidel sweep.  With g = D^-1 r and M = D^-1 B:
//     forward  (ascending i+j):  y_c = g_c - sum_{nb earlier} M_{c,nb} y_nb
//     backward (descending):     x_c = y_c - sum_{nb later}   M_{c,nb} x_nb
// One workgroup walks the hyperplanes h = i + j; thread j owns row j, keeps
// its west / east neighbour in registers and takes the south / north value
// from the neighbouring thread through LDS, so the exact Gauss-Seidel
// dependency order is kept with one barrier per hyperplane.  The wake-cut
// partner (same row 0, earlier or later hyperplane) is kept in LDS.
template <typename T>
__device__ inline void mv_sub(const T *blk, int b, int NS, int s, const T v[4], T out[4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        T a = out[r];
#pragma unroll
        for (int c = 0; c < 4; ++c) a = fma(-blk[BL<T>::at(b, NS, s, r, c)], v[c], a);
        out[r] = a;
    }
}

template <typename T, int BS>
__global__ __launch_bounds__(BS) void k_sgs(BK bk, SweepArgs a) {
    __shared__ T nbuf[2][BS][4];
    extern __shared__ unsigned char smem[];
    LevelDev d;
    if (!take(bk, blockIdx.x, d)) return;
    const Lay L = d.L;
    const T *blk = (const T *)d.blk, *g = (const T *)d.g;
    T *y = (T *)d.y;
    double *xout = a.xout_acc ? d.acc : nullptr;
    double *uu = d.u;
    const double *u0 = d.u0, *dts = d.dts;
    T *row0 = reinterpret_cast<T *>(smem);          // n_wake x 4
    const int j = threadIdx.x;
    const int ni = L.ni, nj = L.nj, NS = L.NS, nw = L.nw;
    const bool active = j < nj;
    const int H = ni + nj - 1;
    // forward sweep
    T yw[4] = {0, 0, 0, 0};
    for (int h = 0; h < H; ++h) {
        const int i = h - j;
        if (active && i >= 0 && i < ni) {
            const int s = L.slot(i, j);
            T v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = g[k * NS + s];
            if (i > 0) mv_sub(blk, B_M0 + 0, NS, s, yw, v);
            if (j > 0) {
                T ys[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) ys[k] = nbuf[(h - 1) & 1][j - 1][k];
                mv_sub(blk, B_M0 + 2, NS, s, ys, v);
            } else if (L.topo == 1 && i >= ni - nw) {
                T yp[4];
                const int p = ni - 1 - i;
#pragma unroll
                for (int k = 0; k < 4; ++k) yp[k] = row0[p * 4 + k];
                mv_sub(blk, B_M0 + 2, NS, s, yp, v);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                nbuf[h & 1][j][k] = v[k];
                y[k * NS + s] = v[k];
                yw[k] = v[k];
            }
            if (j == 0 && L.topo == 1 && i < nw) {
#pragma unroll
                for (int k = 0; k < 4; ++k) row0[i * 4 + k] = v[k];
            }
        }
        lds_barrier();
    }
    // backward sweep (+ stage update); the full barrier completes the y stores
    __syncthreads();
    T xe[4] = {0, 0, 0, 0};
    for (int h = H - 1; h >= 0; --h) {
        const int i = h - j;
        if (active && i >= 0 && i < ni) {
            const int s = L.slot(i, j);
            T v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = y[k * NS + s];
            if (i < ni - 1) mv_sub(blk, B_M0 + 1, NS, s, xe, v);
            if (j == 0 && L.topo == 1 && i < nw) {
                T xp[4];
                const int p = ni - 1 - i - (ni - nw);
#pragma unroll
                for (int k = 0; k < 4; ++k) xp[k] = row0[p * 4 + k];
                mv_sub(blk, B_M0 + 2, NS, s, xp, v);
            }
            if (j < nj - 1) {
                T xn[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) xn[k] = nbuf[(h + 1) & 1][j + 1][k];
                mv_sub(blk, B_M0 + 3, NS, s, xn, v);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                nbuf[h & 1][j][k] = v[k];
                xe[k] = v[k];
            }
            if (j == 0 && L.topo == 1 && i >= ni - nw) {
#pragma unroll
                for (int k = 0; k < 4; ++k) row0[(i - (ni - nw)) * 4 + k] = v[k];
            }
            if (xout) {
#pragma unroll
                for (int k = 0; k < 4; ++k) xout[k * NS + s] = (double)v[k];
            }
            if (a.update) {
                if (a.aw) {
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        uu[k * NS + s] = u0[k * NS + s] - a.alpha * (double)v[k];
                } else {
                    const double dt_s = dts[s];
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        uu[k * NS + s] = u0[k * NS + s] - a.alpha * (dt_s * (double)v[k]);
                }
            }
        }
        lds_barrier();
    }
}

template <typename BT>
__global__ void k_dinv(BK b) {
    const BlockXY cb = xcd_block();
    LevelDev d;
    if (!take(b, cb.y, d)) return;
    const Lay L = d.L;
    const BT *blk = (const BT *)d.blk;
    const double *r = d.F;
    BT *g = (BT *)d.g;
    int s = cb.x * blockDim.x + threadIdx.x;
    int i, j;
    if (!decode(L, s, i, j) || !interior(L, i, j)) return;
    const int NS = L.NS;
    BT rb[4] = {(BT)r[s], (BT)r[NS + s], (BT)r[2 * NS + s], (BT)r[3 * NS + s]};
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        BT a = (BT)0;
#pragma unroll
        for (int c = 0; c < 4; ++c) a = fma(blk[BL<BT>::at(B_DINV, NS, s, rr, c)], rb[c], a);
        g[rr * NS + s] = a;
    }
}

// Same sweeps with four threads per cell row: thread (g, r) owns component
// r of the R consecutive rows j = R g .. R g + R - 1.  Each thread needs one
// row of each 4x4 block per row and hyperplane; these are prefetched into
// registers in two alternating batches of D hyperplanes (load batch B,
// consume batch A, load A, consume B), so each batch is issued D..2D
// hyperplanes before use and every wait only has to exclude the newest
// batch.  A cell of row j on hyperplane h = i + j sits at slot
// (h + 4) NJ + j + 2 of the skewed layout: moving one hyperplane is a
// uniform stride, so every access is a uniform base plus a constant
// per-lane offset.  Neighbour vectors of the previous hyperplane come from
// LDS: every row writes its value every hyperplane (zero where the cell
// does not exist) and zero guard rows sit below row 0 and above the last
// row, so absent neighbours read zero vectors.  One LDS-only barrier per
// hyperplane.
//
// Global memory is accessed through raw buffer resources whose record
// count is the exact extent of the array or plane.  A lane without a cell
// on a hyperplane (before the first column, past the last, or above the
// last row) uses an offset beyond every record count: its loads return
// zeros and its stores are dropped, without touching memory.  Every load
// and store thus stays one unconditional instruction (exact wait counts
// for the prefetch), while absent cells cost no memory traffic.
template <typename T>
__device__ inline T dot4(const T (&m)[4], const T *x) {
    T p0 = fma(m[1], x[1], m[0] * x[0]);
    T p1 = fma(m[3], x[3], m[2] * x[2]);
    return p0 + p1;
}

template <typename T>
__device__ inline T dot4r(const T (&m)[4], const T (&x)[4]) {
    T p0 = fma(m[1], x[1], m[0] * x[0]);
    T p1 = fma(m[3], x[3], m[2] * x[2]);
    return p0 + p1;
}

// a row's 4-vector from LDS (16-byte aligned): two 16-byte reads for FP64,
// one for FP32, so the neighbour rows of a step arrive in one round trip
template <typename T> struct LdsRow;
template <> struct LdsRow<double> {
    __device__ static void get(const double *p, double (&o)[4]) {
        const double2 a = *reinterpret_cast<const double2 *>(p);
        const double2 b = *reinterpret_cast<const double2 *>(p + 2);
        o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
    }
};
template <> struct LdsRow<float> {
    __device__ static void get(const float *p, float (&o)[4]) {
        const float4 a = *reinterpret_cast<const float4 *>(p);
        o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
    }
};

typedef __amdgpu_buffer_rsrc_t Res;
typedef unsigned int U32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int U32x4 __attribute__((ext_vector_type(4)));
constexpr unsigned OOB = 0x80000000u;      // above every record count (extents < 2 GiB)
constexpr int RES_WORD3 = 0x00020000;      // raw (untyped) access, 32-bit data format

__device__ inline Res mkres(const void *p, size_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, RES_WORD3);
}

__device__ inline double bld_d(Res r, unsigned off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ inline void bst_d(Res r, unsigned off, double x) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U32x2, x), r, off, 0, 0);
}

// one value, and one block row of the lane's cell (FP64: 16 bytes from each
// of the two half planes; FP32: the 16-byte row).  The uniform byte offset
// of a block plane goes into the scalar offset: a lane inside the array
// stays inside it, and an out-of-range lane stays out of range (plane
// offsets are below 2^31, so the sum does not wrap).
template <typename T> struct BufIO;
template <> struct BufIO<double> {
    __device__ static double ld(Res r, unsigned off) { return bld_d(r, off); }
    __device__ static void st(Res r, unsigned off, double x) { bst_d(r, off, x); }
    __device__ static void row(Res rb, unsigned off, int p0, int p1, double (&o)[4]) {
        const U32x4 a = __builtin_amdgcn_raw_buffer_load_b128(rb, off, p0, 0);
        const U32x4 b = __builtin_amdgcn_raw_buffer_load_b128(rb, off, p1, 0);
        const double2 da = __builtin_bit_cast(double2, a), db = __builtin_bit_cast(double2, b);
        o[0] = da.x; o[1] = da.y; o[2] = db.x; o[3] = db.y;
    }
};
template <> struct BufIO<float> {
    __device__ static float ld(Res r, unsigned off) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    }
    __device__ static void st(Res r, unsigned off, float x) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, off, 0, 0);
    }
    __device__ static void row(Res rb, unsigned off, int p0, int, float (&o)[4]) {
        const float4 a = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rb, off, p0, 0));
        o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
    }
};

// Row bands (BANDED): the rows of a grid are split into bands of NR rows,
// one workgroup each, so that one grid's sweep runs on several CUs.  Band b
// needs, on hyperplane h, the value of the last row of band b - 1 on
// hyperplane h - 1 (forward) or of the first row of band b + 1 on h + 1
// (backward).  The producing row writes its value of every hyperplane to
// its slot of the hand-off array; the consuming row prefetches it with the
// blocks, waits (bounded) while it still reads the sentinel, puts it into
// its LDS guard row and restores the sentinel.  Every slot written in a
// launch is consumed in it, so between launches the array holds only
// sentinels whatever the band layout.  Hand-off accesses are device-scope
// coherent (bands of one grid may run on different XCDs).  A band waits
// only for its neighbours, which the launcher keeps co-resident; a wait
// that does not end within the spin budget leaves the sentinel (a NaN) in
// the result, so the residual reports divergence instead of a hang: each
// consuming lane has a budget of polls for the whole launch (a correct
// launch needs a few thousand at most), after which it no longer waits.
constexpr int SC1 = 16;                   // cache policy: device-scope coherent
constexpr unsigned BND_SPIN_BUDGET = 1u << 20;

template <typename T> struct Sent;
template <> struct Sent<double> {
    __device__ static bool is(double x) { return __builtin_bit_cast(unsigned long long, x) == BND_SENTINEL64; }
    __device__ static double value() { return __builtin_bit_cast(double, BND_SENTINEL64); }
    __device__ static double ld(Res r, unsigned off) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, SC1));
    }
    __device__ static void st(Res r, unsigned off, double x) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U32x2, x), r, off, 0, SC1);
    }
};
template <> struct Sent<float> {
    __device__ static bool is(float x) { return __builtin_bit_cast(unsigned, x) == BND_SENTINEL32; }
    __device__ static float value() { return __builtin_bit_cast(float, BND_SENTINEL32); }
    __device__ static float ld(Res r, unsigned off) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, SC1));
    }
    __device__ static void st(Res r, unsigned off, float x) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, off, 0, SC1);
    }
};

// the hand-off value prefetched for this hyperplane, once it is written.
// Lanes without the consumer role read zeros (out-of-range offset), so one
// ballot detects the rare step whose consumer still reads the sentinel and
// the spin stays off the common path.
template <typename T>
__device__ inline T bnd_wait(T v, Res r, unsigned off, unsigned &budget) {
    if (__builtin_amdgcn_ballot_w64(Sent<T>::is(v)) != 0) {
        while (Sent<T>::is(v) && budget > 0) {
            __builtin_amdgcn_s_sleep(1);
            v = Sent<T>::ld(r, off);
            --budget;
        }
    }
    return v;
}

// End of a hyperplane step.  A workgroup of one wave needs no barrier: LDS
// instructions of a wave execute in order, so the next step's reads see
// this step's writes once the compiler keeps them in program order.
template <int NT>
__device__ inline void step_sync() {
    if constexpr (NT == 64) __builtin_amdgcn_wave_barrier();
    else lds_barrier();
}

template <typename T, int NT, int R, int D, bool BANDED>
__global__ __launch_bounds__(NT) void k_sgs4(BK bk, SweepArgs a) {
    constexpr int NR = NT / 4 * R;            // rows handled by the workgroup
    constexpr int XS = 4 * NR + 8;            // guard row at both ends
    __shared__ __attribute__((aligned(16))) T xb[2][XS];
    __shared__ T sink[NT];                    // guard-row and wake-row writes of lanes without that role
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    LevelDev dv;
    const int nbands = BANDED ? a.bands : 1;
    const int band = BANDED ? (int)blockIdx.x % nbands : 0;
    // the longest hyperplane chains first: workgroups are placed on CUs in
    // turn, so a long chain's bands share their CUs with bands of shorter
    // cases, which finish early
    const int cidx = BANDED ? (int)blockIdx.x / nbands : (int)blockIdx.x;
    if (!take(bk, bk.order != nullptr ? bk.order[cidx] : cidx, dv)) return;
    const Lay L = dv.L;
    const int ni = L.ni, nj = L.nj, NS = L.NS, NJ = L.NJ, nw = L.nw;
    const int j0 = band * NR;                 // first row of the band
    if (BANDED && j0 >= nj) return;           // band above this case's grid
    const bool below = BANDED && band > 0;                // a band below feeds the forward sweep
    const bool above = BANDED && j0 + NR < nj;            // a band above feeds the backward sweep
    const T *blk = (const T *)dv.blk;
    T *row0 = reinterpret_cast<T *>(smem);                 // n_wake x 4
    T *pblk = row0 + (L.nw > 0 ? L.nw : 1) * 4;           // n_wake x 16: slot-2 blocks of (i, 0), i < n_wake
    const int t = threadIdx.x, grp = t >> 2, r = t & 3;
    const bool cutg = L.topo == 1 && j0 == 0;
    const int H = ni + nj - 1;
    for (int q = t; q < XS; q += NT) {
        xb[0][q] = (T)0;
        xb[1][q] = (T)0;
    }
    if (cutg) {
        for (int q = t; q < nw * 16; q += NT) {
            const int ii = q >> 4, e = q & 15;
            pblk[q] = blk[BL<T>::at(B_M0 + 2, NS, L.slot(ii, 0), e >> 2, e & 3)];
        }
    }
    // resources: the block array (block b, FP64 half plane hf, at a uniform
    // byte offset) and the four-component vectors
    const size_t bstride = (size_t)NS * 16;                // one block (both FP64 half planes)
    const size_t hpl = sizeof(T) == 8 ? (size_t)NS * 8 : 0;  // FP64 second half plane
    const int rec = sizeof(T) == 8 ? 8 : 16;               // values per cell in a plane
    const Res rb = mkres(blk, (size_t)BLK_NBLOCKS * bstride * sizeof(T));
    auto poff = [&](int b, int hf) { return (int)(((size_t)b * bstride + hf * hpl) * sizeof(T)); };
    const size_t vbytes = (size_t)4 * NS * sizeof(T), dbytes = (size_t)4 * NS * sizeof(double);
    const Res rh = mkres(BANDED ? dv.bnd : dv.y, BANDED ? bnd_count(L) * sizeof(T) : 0);
    // per-lane byte offsets at slot base 0 (a hyperplane adds (h + 4) NJ slots)
    unsigned ov[R], ob[R], od[R];
    int jq[R], jx[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        jq[q] = j0 + grp * R + q;
        jx[q] = jq[q] < nj ? jq[q] : jq[q] + (1 << 30);     // rows above the grid never have a cell
        const int jr = jq[q] < nj ? jq[q] : 0;
        ov[q] = (unsigned)((r * NS + jr + NG) * sizeof(T));
        ob[q] = (unsigned)((BL<T>::at(0, NS, jr + NG, r, 0)) * sizeof(T));
        od[q] = (unsigned)((r * NS + jr + NG) * sizeof(double));
    }
    // the lane's cell of row q on hyperplane h exists
    auto cell = [&](int h, int q) { return (unsigned)(h - jx[q]) < (unsigned)ni; };
    // Absent cells (before the first column, past the last, above the last
    // row, padded steps) load zero g (y) and blocks, so their value is +0
    // exactly while the neighbour values are finite: it is written to LDS
    // and handed on as it is, without a select.
    // hand-off lanes: the first row of the band (forward consumer, backward
    // producer) and its last row (forward producer, backward consumer).  A
    // hand-off offset is the uniform part of hyperplane h plus a per-lane
    // part that is out of range on lanes without that role.
    const bool first = grp == 0, last = grp == NT / 4 - 1;
    const int HB = bnd_hb(L);
    auto hrow = [&](bool on, int j) { return on ? (unsigned)((r * HB * NJ + j) * sizeof(T)) : OOB; };
    auto hplane = [&](int h) { return (unsigned)((h + BND_HOFF) * NJ * sizeof(T)); };
    unsigned budget = BND_SPIN_BUDGET;
    // hand-off values wait in a ring of 2D registers, slot = step mod 2D,
    // each loaded P steps before it is needed (short, so that neighbouring
    // bands run only a few steps apart)
    // (banded launches run every step of the last batch: steps past the
    // last hyperplane touch memory only through out-of-range offsets, and
    // unconditional steps keep the compiler's wait counts exact)
    constexpr int NRING = BANDED ? 2 * D : 1;
    constexpr int P = 2 * D - 1 < 3 ? 2 * D - 1 : 3;
    T ring[NRING];
    // ---------------- forward
    {
        const Res rg = mkres(dv.g, vbytes), ry = mkres(dv.y, vbytes);
        const int pw0 = poff(B_M0 + 0, 0), pw1 = poff(B_M0 + 0, 1);
        const int ps0 = poff(B_M0 + 2, 0), ps1 = poff(B_M0 + 2, 1);
        const bool cons = below && first, prod = above && last;
        const unsigned hl = hrow(cons, j0 - 1), hs = cons ? hl : hrow(prod, j0 + NR - 1);
        T gA[D][R], wA[D][R][4], sA[D][R][4], gB[D][R], wB[D][R][4], sB[D][R][4];
        auto load = [&](T (&gg)[D][R], T (&ww)[D][R][4], T (&ss)[D][R][4], int hb) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const int h = hb + k;
                const unsigned hv = (unsigned)((h + 2 * NG) * NJ);
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const bool ok = cell(h, q);
                    const unsigned og = ok ? hv * (unsigned)sizeof(T) + ov[q] : OOB;
                    const unsigned obk = ok ? hv * (unsigned)(rec * sizeof(T)) + ob[q] : OOB;
                    gg[k][q] = BufIO<T>::ld(rg, og);
                    BufIO<T>::row(rb, obk, pw0, pw1, ww[k][q]);
                    BufIO<T>::row(rb, obk, ps0, ps1, ss[k][q]);
                }
            }
        };
        // consumer lanes put the hand-off value into the guard row of the
        // next hyperplane's buffer, the other lanes into their sink slot
        T *const gd[2] = {cons ? &xb[0][r] : &sink[t], cons ? &xb[1][r] : &sink[t]};
        // step sl of a batch (h0 + sl = h, h0 even): buffers alternate with sl
        auto step = [&](auto wake, const T (&gv)[R], const T (&wv)[R][4], const T (&sv)[R][4], int sl, int h) {
            constexpr bool WAKE = decltype(wake)::value;
            const T *prev = xb[(sl + 1) & 1];
            T *cur = xb[sl & 1];
            const unsigned hv = (unsigned)((h + 2 * NG) * NJ);
            if constexpr (BANDED) {
                // the row below the band on this hyperplane, for the next one
                *gd[sl & 1] = bnd_wait(ring[sl], rh, hplane(h) + hl, budget);
                ring[(sl + P) % NRING] = Sent<T>::ld(rh, hplane(h + P) + hl);
            }
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int jj = jq[q] - j0;                          // row within the band
                const T *xs = prev + 4 * jj;                        // row below (guard row for jj = 0)
                // Wake-cut code is branch-free: lane- and step-dependent
                // choices are selects (a branch here costs the compiler its
                // count of the prefetch loads in flight, and every later step
                // of the batch then waits for them).
                if constexpr (WAKE) {                               // row 0 at i = h: wake-cut partner
                    const bool part = jq[q] == 0 && h >= ni - nw && h < ni;
                    xs = part ? row0 + (ni - 1 - h) * 4 : xs;
                }
                T xw[4], xsv[4];
                LdsRow<T>::get(prev + 4 * jj + 4, xw);
                LdsRow<T>::get(xs, xsv);
                const T v = (gv[q] - dot4r(wv[q], xw)) - dot4r(sv[q], xsv);
                cur[4 * jj + 4 + r] = v;
                BufIO<T>::st(ry, cell(h, q) ? hv * (unsigned)sizeof(T) + ov[q] : OOB, v);
                if constexpr (WAKE) {
                    const bool keep = jq[q] == 0 && h < nw;
                    *(keep ? row0 + h * 4 + r : &sink[t]) = v;
                }
                // one store: the last row's value (producer lanes) and the
                // sentinel back into the slot just consumed (consumer lanes)
                if constexpr (BANDED)
                    if (q == R - 1)
                        Sent<T>::st(rh, hplane(h) + hs, cons ? Sent<T>::value() : v);
            }
            step_sync<NT>();
        };
        if constexpr (BANDED) {
#pragma unroll
            for (int k = 0; k < P; ++k) ring[k] = Sent<T>::ld(rh, hplane(k) + hl);
        }
        // a batch of 2D hyperplanes; the wake-cut code is compiled only into
        // the variant that band 0 of a C-grid runs near the cut columns
        auto batch = [&](auto wake, int h0) {
            load(gB, wB, sB, h0 + D);
#pragma unroll
            for (int k = 0; k < D; ++k)
                if (BANDED || h0 + k < H) step(wake, gA[k], wA[k], sA[k], k, h0 + k);
            load(gA, wA, sA, h0 + 2 * D);
#pragma unroll
            for (int k = 0; k < D; ++k)
                if (BANDED || h0 + D + k < H) step(wake, gB[k], wB[k], sB[k], D + k, h0 + D + k);
        };
        load(gA, wA, sA, 0);
        __syncthreads();
        for (int h0 = 0; h0 < H; h0 += 2 * D) {
            // row 0 of the batch's hyperplanes outside [0, nw) and [ni - nw, ni)
            const bool plain = !cutg || h0 >= ni || (h0 >= nw && h0 + 2 * D <= ni - nw);
            if (plain) batch(std::false_type(), h0);
            else batch(std::true_type(), h0);
        }
    }
    // ---------------- backward (+ stage update); the full barrier completes the y stores
    __syncthreads();
    for (int q = t; q < XS; q += NT) {
        xb[0][q] = (T)0;
        xb[1][q] = (T)0;
    }
    __syncthreads();
    {
        const Res ry = mkres(dv.y, vbytes);
        const int pe0 = poff(B_M0 + 1, 0), pe1 = poff(B_M0 + 1, 1);
        const int pn0 = poff(B_M0 + 3, 0), pn1 = poff(B_M0 + 3, 1);
        const Res ru0 = mkres(a.update ? dv.u0 : dv.u, dbytes), ruu = mkres(dv.u, dbytes);
        const Res rx = mkres(dv.acc, dbytes);
        const Res rdt = mkres(dv.dts, (size_t)NS * sizeof(double));
        const bool cons = above && last, prod = below && first;
        const unsigned hl = hrow(cons, j0 + NR), hs = cons ? hl : hrow(prod, j0);
        T yA[D][R], eA[D][R][4], nA[D][R][4], yB[D][R], eB[D][R][4], nB[D][R][4];
        double uA[D][R], uB[D][R], tA[D][R], tB[D][R];
        const bool want_dt = a.update && !a.aw;
        auto load = [&](T (&yy)[D][R], T (&ee)[D][R][4], T (&nn)[D][R][4], double (&u0r)[D][R], double (&dtr)[D][R],
                        int hb) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const int h = H - 1 - (hb + k);
                const unsigned hv = (unsigned)((h + 2 * NG) * NJ);
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const bool ok = cell(h, q);
                    const unsigned obk = ok ? hv * (unsigned)(rec * sizeof(T)) + ob[q] : OOB;
                    yy[k][q] = BufIO<T>::ld(ry, ok ? hv * (unsigned)sizeof(T) + ov[q] : OOB);
                    u0r[k][q] = bld_d(ru0, ok && a.update ? hv * 8u + od[q] : OOB);
                    dtr[k][q] = bld_d(rdt, ok && want_dt ? (hv + (unsigned)(jq[q] + NG)) * 8u : OOB);
                    BufIO<T>::row(rb, obk, pe0, pe1, ee[k][q]);
                    BufIO<T>::row(rb, obk, pn0, pn1, nn[k][q]);
                }
            }
        };
        T *const gd[2] = {cons ? &xb[0][4 * NR + 4 + r] : &sink[t], cons ? &xb[1][4 * NR + 4 + r] : &sink[t]};
        // step sl of a batch: buffers alternate with the step
        auto step = [&](auto wake, const T (&yv)[R], const T (&ev)[R][4], const T (&nv)[R][4],
                        const double (&u0v)[R], const double (&dtv)[R], const T (&wz)[R], int sl, int h) {
            constexpr int WK = decltype(wake)::value;
            const T *prev = xb[(sl + 1) & 1];
            T *cur = xb[sl & 1];
            const unsigned hv = (unsigned)((h + 2 * NG) * NJ);
            if constexpr (BANDED) {
                // the row above the band on this hyperplane, for the next one
                *gd[sl & 1] = bnd_wait(ring[sl], rh, hplane(h) + hl, budget);
                ring[(sl + P) % NRING] = Sent<T>::ld(rh, hplane(h - P) + hl);
            }
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int jj = jq[q] - j0;
                T xe[4], xn[4];
                LdsRow<T>::get(prev + 4 * jj + 4, xe);
                LdsRow<T>::get(prev + 4 * jj + 8, xn);
                T v = (yv[q] - dot4r(ev[q], xe)) - dot4r(nv[q], xn);
                if constexpr (WK == 1) {                           // row 0 at i = h: wake-cut partner
                    v = jq[q] == 0 && h >= 0 && h < nw ? v - wz[q] : v;
                } else if constexpr (WK == 2) {
                    if (h >= 0 && h < nw && jq[q] == 0) {
                        T mp[4];
#pragma unroll
                        for (int c = 0; c < 4; ++c) mp[c] = pblk[h * 16 + r * 4 + c];
                        v = v - dot4(mp, row0 + (nw - 1 - h) * 4);
                    }
                }
                const bool valid = cell(h, q);
                cur[4 * jj + 4 + r] = v;
                if constexpr (WK != 0) {
                    const bool keep = jq[q] == 0 && h >= ni - nw && h < ni;
                    *(keep ? row0 + (h - (ni - nw)) * 4 + r : &sink[t]) = v;
                }
                if constexpr (BANDED)
                    if (q == 0)
                        Sent<T>::st(rh, hplane(h) + hs, cons ? Sent<T>::value() : v);
                const unsigned oe = valid ? hv * 8u + od[q] : OOB;
                if (a.xout_acc) bst_d(rx, oe, (double)v);
                if (a.update) {
                    double un;
                    if (a.aw) un = u0v[q] - a.alpha * (double)v;
                    else un = u0v[q] - a.alpha * (dtv[q] * (double)v);
                    bst_d(ruu, oe, un);
                }
            }
            step_sync<NT>();
        };
        if constexpr (BANDED) {
#pragma unroll
            for (int k = 0; k < P; ++k) ring[k] = Sent<T>::ld(rh, hplane(H - 1 - k) + hl);
        }
        // Partner terms of the row-0 wake cells of the D hyperplanes from
        // backward position hb on (hyperplanes H - 1 - hb downwards), formed
        // before the steps when every partner (hyperplane ni - 1 - h, at least
        // ni - nw) lies above them, i.e. was swept in an earlier batch: the
        // step then subtracts a register instead of waiting on two LDS reads
        // and four products on its chain (the same operations in the same
        // order, so the same value).
        // (variant 1; clamped addresses, so that no lane branches)
        auto wake_terms = [&](auto wake, T (&wz)[D][R], int hb) {
            constexpr int WK = decltype(wake)::value;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const int h = H - 1 - (hb + k);
                const bool in = h >= 0 && h < nw;
                const int hw = in ? h : 0;
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    T z = (T)0;
                    if constexpr (WK == 1) {
                        T mp[4];
#pragma unroll
                        for (int c = 0; c < 4; ++c) mp[c] = pblk[hw * 16 + r * 4 + c];
                        z = dot4(mp, row0 + (in ? nw - 1 - h : 0) * 4);
                    }
                    wz[k][q] = z;
                }
            }
        };
        T wz[D][R];
        auto batch = [&](auto wake, int h0) {
            load(yB, eB, nB, uB, tB, h0 + D);
            wake_terms(wake, wz, h0);
#pragma unroll
            for (int k = 0; k < D; ++k)
                if (BANDED || h0 + k < H) step(wake, yA[k], eA[k], nA[k], uA[k], tA[k], wz[k], k, H - 1 - (h0 + k));
            load(yA, eA, nA, uA, tA, h0 + 2 * D);
            wake_terms(wake, wz, h0 + D);
#pragma unroll
            for (int k = 0; k < D; ++k)
                if (BANDED || h0 + D + k < H)
                    step(wake, yB[k], eB[k], nB[k], uB[k], tB[k], wz[k], D + k, H - 1 - (h0 + D + k));
        };
        load(yA, eA, nA, uA, tA, 0);
        __syncthreads();
        for (int h0 = 0; h0 < H; h0 += 2 * D) {
            // the batch's hyperplanes H - 1 - h0 down to H - 2D - h0
            const int hhi = H - 1 - h0, hlo = H - 2 * D - h0;
            const bool plain = !cutg || hlo >= ni || hhi < 0 || (hlo >= nw && hhi < ni - nw);
            // variant 1 when every wake partner of the batch (hyperplanes from
            // ni - nw up) was swept in an earlier batch
            if (plain) batch(std::integral_constant<int, 0>(), h0);
            else if (ni - nw > hhi) batch(std::integral_constant<int, 1>(), h0);
            else batch(std::integral_constant<int, 2>(), h0);
        }
    }
}

// Eight threads per cell row (k_sgs8): thread t = 8 g + 2 rr + hf of the
// band's row g computes block row rr over the columns 2 hf and 2 hf + 1 of
// each block: its half of the product, fma(m1, x1, m0 x0) or
// fma(m3, x3, m2 x2), is exactly one of the two halves k_sgs4 adds, and the
// lanes t and t ^ 1 exchange their halves with one DPP swap and add them in
// either order (a + b = b + a exactly), so both lanes hold the row's value
// bitwise as k_sgs4 forms it.  A lane's memory per hyperplane is one value
// and one 16-byte (FP32: 8-byte) half row of each block, half of what a
// four-thread lane moves, and its instruction stream per step is about half
// as long; the band's rows are spread over NW waves of eight rows, which
// meet at an LDS barrier after every step.  Layout, prefetch batches,
// out-of-range offsets for absent cells, the hand-off between row bands
// and the wake-cut coupling are those of k_sgs4.
template <typename T> struct Half;
template <> struct Half<double> {
    // the two values of a half row: one 16-byte load
    __device__ static void ld(Res r, unsigned off, int plane, double (&o)[2]) {
        const double2 a = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, plane, 0));
        o[0] = a.x;
        o[1] = a.y;
    }
    __device__ static void lds(const double *p, double (&o)[2]) {
        const double2 a = *reinterpret_cast<const double2 *>(p);
        o[0] = a.x;
        o[1] = a.y;
    }
    // the partner lane's value (lanes t and t ^ 1: quad permutation 1 0 3 2)
    __device__ static double swap(double x) {
        const U32x2 v = __builtin_bit_cast(U32x2, x);
        U32x2 o;
        o.x = (unsigned)__builtin_amdgcn_mov_dpp((int)v.x, 0xB1, 0xF, 0xF, false);
        o.y = (unsigned)__builtin_amdgcn_mov_dpp((int)v.y, 0xB1, 0xF, 0xF, false);
        return __builtin_bit_cast(double, o);
    }
};
template <> struct Half<float> {
    __device__ static void ld(Res r, unsigned off, int plane, float (&o)[2]) {
        // the whole result is bit-cast to a full-width type: element access
        // on the builtin's own vector type reads element 0 twice here
        const float2 a = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, plane, 0));
        o[0] = a.x;
        o[1] = a.y;
    }
    __device__ static void lds(const float *p, float (&o)[2]) {
        const float2 a = *reinterpret_cast<const float2 *>(p);
        o[0] = a.x;
        o[1] = a.y;
    }
    __device__ static float swap(float x) {
        return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0xB1, 0xF, 0xF, false));
    }
};

template <typename T>
__device__ inline T half_dot(const T (&m)[2], const T (&x)[2]) {
    return fma(m[1], x[1], m[0] * x[0]);
}

template <typename T, int NW, int D, bool BANDED>
__global__ __launch_bounds__(64 * NW) void k_sgs8(BK bk, SweepArgs a) {
    constexpr int NT = 64 * NW;
    constexpr int NR = 8 * NW;                // rows handled by the workgroup
    constexpr int XS = 4 * NR + 8;            // guard row at both ends
    __shared__ __attribute__((aligned(16))) T xb[2][XS];
    __shared__ T sink[NT];                    // guard-row and wake-row writes of lanes without that role
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    LevelDev dv;
    const int nbands = BANDED ? a.bands : 1;
    const int band = BANDED ? (int)blockIdx.x % nbands : 0;
    // the longest hyperplane chains first: workgroups are placed on CUs in
    // turn, so a long chain's bands share their CUs with bands of shorter
    // cases, which finish early
    const int cidx = BANDED ? (int)blockIdx.x / nbands : (int)blockIdx.x;
    if (!take(bk, bk.order != nullptr ? bk.order[cidx] : cidx, dv)) return;
    const Lay L = dv.L;
    const int ni = L.ni, nj = L.nj, NS = L.NS, NJ = L.NJ, nw = L.nw;
    const int j0 = band * NR;
    if (BANDED && j0 >= nj) return;
    const bool below = BANDED && band > 0;
    const bool above = BANDED && j0 + NR < nj;
    const T *blk = (const T *)dv.blk;
    T *row0 = reinterpret_cast<T *>(smem);                 // n_wake x 4
    T *pblk = row0 + (L.nw > 0 ? L.nw : 1) * 4;           // n_wake x 16: slot-2 blocks of (i, 0), i < n_wake
    const int t = threadIdx.x, grp = t >> 3, rr = (t >> 1) & 3, hf = t & 1;
    const bool cutg = L.topo == 1 && j0 == 0;
    const int H = ni + nj - 1;
    for (int q = t; q < XS; q += NT) {
        xb[0][q] = (T)0;
        xb[1][q] = (T)0;
    }
    if (cutg) {
        for (int q = t; q < nw * 16; q += NT) {
            const int ii = q >> 4, e = q & 15;
            pblk[q] = blk[BL<T>::at(B_M0 + 2, NS, L.slot(ii, 0), e >> 2, e & 3)];
        }
    }
    const size_t bstride = (size_t)NS * 16;
    const int rec = sizeof(T) == 8 ? 8 : 16;               // values per cell in a plane
    const Res rb = mkres(blk, (size_t)BLK_NBLOCKS * bstride * sizeof(T));
    auto poff = [&](int b) { return (int)((size_t)b * bstride * sizeof(T)); };
    const size_t vbytes = (size_t)4 * NS * sizeof(T), dbytes = (size_t)4 * NS * sizeof(double);
    const Res rh = mkres(BANDED ? dv.bnd : dv.y, BANDED ? bnd_count(L) * sizeof(T) : 0);
    // per-lane byte offsets at slot base 0 (a hyperplane adds (h + 4) NJ slots);
    // the half row of block 0 at this lane's row, row rr and columns 2 hf ..
    const int jq = j0 + grp;
    const int jx = jq < nj ? jq : jq + (1 << 30);          // rows above the grid never have a cell
    const int jr = jq < nj ? jq : 0;
    const unsigned ov = (unsigned)((rr * NS + jr + NG) * sizeof(T));
    const unsigned ob = (unsigned)(BL<T>::at(0, NS, jr + NG, rr, 2 * hf) * sizeof(T));
    const unsigned od = (unsigned)((rr * NS + jr + NG) * sizeof(double));
    const bool lead = hf == 0;                             // the lane of the pair that stores
    auto cell = [&](int h) { return (unsigned)(h - jx) < (unsigned)ni; };
    const bool first = grp == 0, last = grp == NR - 1;
    const int HB = bnd_hb(L);
    auto hrow = [&](bool on, int j) { return on ? (unsigned)((rr * HB * NJ + j) * sizeof(T)) : OOB; };
    auto hplane = [&](int h) { return (unsigned)((h + BND_HOFF) * NJ * sizeof(T)); };
    unsigned budget = BND_SPIN_BUDGET;
    constexpr int NRING = BANDED ? 2 * D : 1;
    constexpr int P = 2 * D - 1 < 3 ? 2 * D - 1 : 3;
    T ring[NRING];
    const int jj = jq - j0;                                // row within the band
    // ---------------- forward
    {
        const Res rg = mkres(dv.g, vbytes), ry = mkres(dv.y, vbytes);
        const int pw = poff(B_M0 + 0), ps = poff(B_M0 + 2);
        const bool cons = below && first && lead, prod = above && last && lead;
        const unsigned hl = hrow(cons, j0 - 1), hs = cons ? hl : hrow(prod, j0 + NR - 1);
        T gA[D], wA[D][2], sA[D][2], gB[D], wB[D][2], sB[D][2];
        auto load = [&](T (&gg)[D], T (&ww)[D][2], T (&ss)[D][2], int hb) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const int h = hb + k;
                const unsigned hv = (unsigned)((h + 2 * NG) * NJ);
                const bool ok = cell(h);
                gg[k] = BufIO<T>::ld(rg, ok ? hv * (unsigned)sizeof(T) + ov : OOB);
                const unsigned obk = ok ? hv * (unsigned)(rec * sizeof(T)) + ob : OOB;
                Half<T>::ld(rb, obk, pw, ww[k]);
                Half<T>::ld(rb, obk, ps, ss[k]);
            }
        };
        T *const gd[2] = {cons ? &xb[0][rr] : &sink[t], cons ? &xb[1][rr] : &sink[t]};
        auto step = [&](auto wake, const T gv, const T (&wv)[2], const T (&sv)[2], int sl, int h) {
            constexpr bool WAKE = decltype(wake)::value;
            const T *prev = xb[(sl + 1) & 1];
            T *cur = xb[sl & 1];
            const unsigned hv = (unsigned)((h + 2 * NG) * NJ);
            if constexpr (BANDED) {
                *gd[sl & 1] = bnd_wait(ring[sl], rh, hplane(h) + hl, budget);
                ring[(sl + P) % NRING] = Sent<T>::ld(rh, hplane(h + P) + hl);
            }
            const T *xs = prev + 4 * jj + 2 * hf;                  // row below (guard row for jj = 0)
            if (WAKE && h >= ni - nw && h < ni) {                  // row 0 at i = h: wake-cut partner
                xs = jq == 0 ? row0 + (ni - 1 - h) * 4 + 2 * hf : xs;
            }
            T xw[2], xsv[2];
            Half<T>::lds(prev + 4 * jj + 4 + 2 * hf, xw);
            Half<T>::lds(xs, xsv);
            const T pw_ = half_dot(wv, xw), ps_ = half_dot(sv, xsv);
            const T dw = pw_ + Half<T>::swap(pw_), ds = ps_ + Half<T>::swap(ps_);
            const T v = (gv - dw) - ds;
            cur[4 * jj + 4 + rr] = v;
            BufIO<T>::st(ry, cell(h) && lead ? hv * (unsigned)sizeof(T) + ov : OOB, v);
            if (WAKE && h < nw) *(jq == 0 ? row0 + h * 4 + rr : &sink[t]) = v;
            if constexpr (BANDED) Sent<T>::st(rh, hplane(h) + hs, cons ? Sent<T>::value() : v);
            step_sync<NT>();
        };
        if constexpr (BANDED) {
#pragma unroll
            for (int k = 0; k < P; ++k) ring[k] = Sent<T>::ld(rh, hplane(k) + hl);
        }
        auto batch = [&](auto wake, int h0) {
            load(gB, wB, sB, h0 + D);
#pragma unroll
            for (int k = 0; k < D; ++k)
                if (BANDED || h0 + k < H) step(wake, gA[k], wA[k], sA[k], k, h0 + k);
            load(gA, wA, sA, h0 + 2 * D);
#pragma unroll
            for (int k = 0; k < D; ++k)
                if (BANDED || h0 + D + k < H) step(wake, gB[k], wB[k], sB[k], D + k, h0 + D + k);
        };
        load(gA, wA, sA, 0);
        __syncthreads();
        for (int h0 = 0; h0 < H; h0 += 2 * D) {
            const bool plain = !cutg || h0 >= ni || (h0 >= nw && h0 + 2 * D <= ni - nw);
            if (plain) batch(std::false_type(), h0);
            else batch(std::true_type(), h0);
        }
    }
    // ---------------- backward (+ stage update); the full barrier completes the y stores
    __syncthreads();
    for (int q = t; q < XS; q += NT) {
        xb[0][q] = (T)0;
        xb[1][q] = (T)0;
    }
    __syncthreads();
    {
        const Res ry = mkres(dv.y, vbytes);
        const int pe = poff(B_M0 + 1), pn = poff(B_M0 + 3);
        const Res ru0 = mkres(a.update ? dv.u0 : dv.u, dbytes), ruu = mkres(dv.u, dbytes);
        const Res rx = mkres(dv.acc, dbytes);
        const Res rdt = mkres(dv.dts, (size_t)NS * sizeof(double));
        const bool cons = above && last && lead, prod = below && first && lead;
        const unsigned hl = hrow(cons, j0 + NR), hs = cons ? hl : hrow(prod, j0);
        T yA[D], eA[D][2], nA[D][2], yB[D], eB[D][2], nB[D][2];
        double uA[D], uB[D], tA[D], tB[D];
        const bool want_dt = a.update && !a.aw;
        auto load = [&](T (&yy)[D], T (&ee)[D][2], T (&nn)[D][2], double (&u0r)[D], double (&dtr)[D], int hb) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const int h = H - 1 - (hb + k);
                const unsigned hv = (unsigned)((h + 2 * NG) * NJ);
                const bool ok = cell(h);
                const unsigned obk = ok ? hv * (unsigned)(rec * sizeof(T)) + ob : OOB;
                yy[k] = BufIO<T>::ld(ry, ok ? hv * (unsigned)sizeof(T) + ov : OOB);
                u0r[k] = bld_d(ru0, ok && lead && a.update ? hv * 8u + od : OOB);
                dtr[k] = bld_d(rdt, ok && lead && want_dt ? (hv + (unsigned)(jq + NG)) * 8u : OOB);
                Half<T>::ld(rb, obk, pe, ee[k]);
                Half<T>::ld(rb, obk, pn, nn[k]);
            }
        };
        T *const gd[2] = {cons ? &xb[0][4 * NR + 4 + rr] : &sink[t], cons ? &xb[1][4 * NR + 4 + rr] : &sink[t]};
        auto step = [&](auto wake, const T yv, const T (&ev)[2], const T (&nv)[2], const double u0v,
                        const double dtv, int sl, int h) {
            constexpr bool WAKE = decltype(wake)::value;
            const T *prev = xb[(sl + 1) & 1];
            T *cur = xb[sl & 1];
            const unsigned hv = (unsigned)((h + 2 * NG) * NJ);
            if constexpr (BANDED) {
                *gd[sl & 1] = bnd_wait(ring[sl], rh, hplane(h) + hl, budget);
                ring[(sl + P) % NRING] = Sent<T>::ld(rh, hplane(h - P) + hl);
            }
            T xe[2], xn[2];
            Half<T>::lds(prev + 4 * jj + 4 + 2 * hf, xe);
            Half<T>::lds(prev + 4 * jj + 8 + 2 * hf, xn);
            const T pe_ = half_dot(ev, xe), pn_ = half_dot(nv, xn);
            const T de = pe_ + Half<T>::swap(pe_), dn = pn_ + Half<T>::swap(pn_);
            T v = (yv - de) - dn;
            if constexpr (WAKE) {
                // row 0 at i = h < n_wake: the wake-cut partner's term; every
                // lane forms a half product (clamped addresses) so that the
                // swap runs with all lanes, and row 0 keeps it
                const bool wk = h >= 0 && h < nw;
                const int hw = wk ? h : 0;
                T mp[2], xp[2];
                mp[0] = pblk[hw * 16 + rr * 4 + 2 * hf];
                mp[1] = pblk[hw * 16 + rr * 4 + 2 * hf + 1];
                Half<T>::lds(row0 + (wk ? nw - 1 - h : 0) * 4 + 2 * hf, xp);
                const T pp = half_dot(mp, xp);
                const T dp = pp + Half<T>::swap(pp);
                if (wk && jq == 0) v = v - dp;
            }
            const bool valid = cell(h);
            cur[4 * jj + 4 + rr] = v;
            if (WAKE && h >= ni - nw && h < ni) *(jq == 0 ? row0 + (h - (ni - nw)) * 4 + rr : &sink[t]) = v;
            if constexpr (BANDED) Sent<T>::st(rh, hplane(h) + hs, cons ? Sent<T>::value() : v);
            const unsigned oe = valid && lead ? hv * 8u + od : OOB;
            if (a.xout_acc) bst_d(rx, oe, (double)v);
            if (a.update) {
                double un;
                if (a.aw) un = u0v - a.alpha * (double)v;
                else un = u0v - a.alpha * (dtv * (double)v);
                bst_d(ruu, oe, un);
            }
            step_sync<NT>();
        };
        if constexpr (BANDED) {
#pragma unroll
            for (int k = 0; k < P; ++k) ring[k] = Sent<T>::ld(rh, hplane(H - 1 - k) + hl);
        }
        auto batch = [&](auto wake, int h0) {
            load(yB, eB, nB, uB, tB, h0 + D);
#pragma unroll
            for (int k = 0; k < D; ++k)
                if (BANDED || h0 + k < H) step(wake, yA[k], eA[k], nA[k], uA[k], tA[k], k, H - 1 - (h0 + k));
            load(yA, eA, nA, uA, tA, h0 + 2 * D);
#pragma unroll
            for (int k = 0; k < D; ++k)
                if (BANDED || h0 + D + k < H)
                    step(wake, yB[k], eB[k], nB[k], uB[k], tB[k], D + k, H - 1 - (h0 + D + k));
        };
        load(yA, eA, nA, uA, tA, 0);
        __syncthreads();
        for (int h0 = 0; h0 < H; h0 += 2 * D) {
            const int hhi = H - 1 - h0, hlo = H - 2 * D - h0;
            const bool plain = !cutg || hlo >= ni || hhi < 0 || (hlo >= nw && hhi < ni - nw);
            if (plain) batch(std::false_type(), h0);
            else batch(std::true_type(), h0);
        }
    }
}

// ------------------------------------------------------------ transfers
// Section 3: restriction = volume-weighted agglomeration of 2x2 cells.
// Each job restricts the fine-level combination a x (+ b y), formed per
// fine cell as the elementwise update of the same name would form it.
__global__ void k_restrict(BK bf, BK bc, RJob j0, RJob j1, int njobs, int mut) {
    const BlockXY cb = xcd_block();
    LevelDev df, dc;
    if (!take(bf, cb.y, df) || !take(bc, cb.y, dc)) return;
    const Lay Lf = df.L, Lc = dc.L;
    const double *geof = df.geo, *geoc = dc.geo;
    int s = cb.x * blockDim.x + threadIdx.x;
    int i, j;
    if (!decode(Lc, s, i, j) || !interior(Lc, i, j)) return;
    const int NSf = Lf.NS, NSc = Lc.NS;
    int c00 = Lf.slot(2 * i, 2 * j), c10 = Lf.slot(2 * i + 1, 2 * j);
    int c01 = Lf.slot(2 * i, 2 * j + 1), c11 = Lf.slot(2 * i + 1, 2 * j + 1);
    double v00 = geof[G_VOL * NSf + c00], v10 = geof[G_VOL * NSf + c10];
    double v01 = geof[G_VOL * NSf + c01], v11 = geof[G_VOL * NSf + c11];
    double vol = geoc[G_VOL * NSc + s];
    for (int q = 0; q < njobs; ++q) {
        const RJob jb = q == 0 ? j0 : j1;
        const double *x = field(df, jb.fx), *y = field(df, jb.fy);
        double *vc = field(dc, jb.fout), *vc2 = field(dc, jb.fout2);
        auto val = [&](int o) { return y ? jb.a * x[o] + jb.b * y[o] : jb.a * x[o]; };
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double w00 = val(k * NSf + c00) * v00, w10 = val(k * NSf + c10) * v10;
            double w01 = val(k * NSf + c01) * v01, w11 = val(k * NSf + c11) * v11;
            double r = (((w00 + w10) + w01) + w11) / vol;
            vc[k * NSc + s] = r;
            if (vc2) vc2[k * NSc + s] = r;
        }
    }
    if (mut) {
        double w00 = df.mut[c00] * v00, w10 = df.mut[c10] * v10;
        double w01 = df.mut[c01] * v01, w11 = df.mut[c11] * v11;
        dc.mut[s] = (((w00 + w10) + w01) + w11) / vol;
    }
}

// Section 3: bilinear prolongation of the coarse correction, weights
// 9/16 (parent), 3/16, 3/16, 1/16 towards the fine cell's side; the wake-cut
// partner across the cut, the parent's value where a neighbour is missing.
__global__ void k_prolong(BK bf, BK bc) {
    const BlockXY cb = xcd_block();
    LevelDev df, dc;
    if (!take(bf, cb.y, df) || !take(bc, cb.y, dc)) return;
    const Lay Lf = df.L, Lc = dc.L;
    const double *uc = dc.u, *utc = dc.ut;
    double *uf = df.u;
    int s = cb.x * blockDim.x + threadIdx.x;
    int i, j;
    if (!decode(Lf, s, i, j) || !interior(Lf, i, j)) return;
    const int NSc = Lc.NS, NSf = Lf.NS;
    int I = i / 2, J = j / 2;
    int In = I + ((i & 1) ? 1 : -1), Jn = J + ((j & 1) ? 1 : -1);
    bool vi = In >= 0 && In < Lc.ni, vj = Jn >= 0 && Jn < Lc.nj;
    int s0 = Lc.slot(I, J);
    int s1 = vi ? Lc.slot(In, J) : s0;
    int s2 = s0, s3 = s0;
    if (vj) s2 = Lc.slot(I, Jn);
    else if (Jn < 0 && cut_col(Lc, I)) s2 = Lc.slot(Lc.ni - 1 - I, 0);
    if (vi && vj) s3 = Lc.slot(In, Jn);
    else if (vi && Jn < 0 && cut_col(Lc, In)) s3 = Lc.slot(Lc.ni - 1 - In, 0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double e0 = uc[k * NSc + s0] - utc[k * NSc + s0];
        double e1 = uc[k * NSc + s1] - utc[k * NSc + s1];
        double e2 = uc[k * NSc + s2] - utc[k * NSc + s2];
        double e3 = uc[k * NSc + s3] - utc[k * NSc + s3];
        double pe = (((9.0 * e0 + 3.0 * e1) + 3.0 * e2) + e3) * 0.0625;
        uf[k * NSf + s] = uf[k * NSf + s] + pe;
    }
}

// out = a x (+ b y) on the interior cells, fields named per case
__global__ void k_axpby(BK bk, double a, int fx, double b, int fy, int fout) {
    const BlockXY cb = xcd_block();
    LevelDev d;
    if (!take(bk, cb.y, d)) return;
    const Lay L = d.L;
    const double *x = field(d, fx), *y = field(d, fy);
    double *out = field(d, fout);
    int s = cb.x * blockDim.x + threadIdx.x;
    int i, j;
    if (!decode(L, s, i, j) || !interior(L, i, j)) return;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int o = k * L.NS + s;
        out[o] = (y == nullptr) ? a * x[o] : a * x[o] + b * y[o];
    }
}

// roll-back of a diverged cycle: u = ulast on the interior cells of every
// case flagged by the status update (the activity flag is already 0)
__global__ void k_rollback(BK bk, const int *rb) {
    if (rb[blockIdx.y] == 0) return;
    const LevelDevG &g = reinterpret_cast<const LevelDevG *>(bk.V)[blockIdx.y];
    const Lay L = g.L;
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    int i, j;
    if (!decode(L, s, i, j) || !interior(L, i, j)) return;
#pragma unroll
    for (int k = 0; k < 4; ++k) g.u[k * L.NS + s] = g.ulast[k * L.NS + s];
}

__global__ void k_pack(Lay L, const double *p, double *n, int nc) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int N = L.ni * L.nj;
    if (t >= N) return;
    int j = t / L.ni, i = t - j * L.ni;
    int s = L.slot(i, j);
    for (int k = 0; k < nc; ++k) n[k * N + t] = p[k * L.NS + s];
}

__global__ void k_unpack(Lay L, const double *n, double *p, int nc) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int N = L.ni * L.nj;
    if (t >= N) return;
    int j = t / L.ni, i = t - j * L.ni;
    int s = L.slot(i, j);
    for (int k = 0; k < nc; ++k) p[k * L.NS + s] = n[k * N + t];
}

// RMS of the density component of F over interior cells; fixed-order
// two-pass reduction (deterministic).
constexpr int RED_BLOCKS = 128;
// RMS of the fine residual's first component over the interior: each
// thread sums a strided share of the interior cells (hyperplane order, so a
// wave's loads are consecutive slots), the wave adds its lanes by butterfly
// shuffles, and lane 0's sum of the workgroup's waves (in wave order) is its
// partial; k_norm2 adds the partials the same way.  Every order is fixed,
// so the norm does not depend on scheduling.
__global__ __launch_bounds__(TPB) void k_norm1(BK bk) {
    __shared__ double sh[TPB / 64];
    LevelDev d;
    if (!take(bk, blockIdx.y, d)) return;
    const Lay L = d.L;
    const double *F = d.F;
    const int n = L.ni * L.nj;
    double a = 0.0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        int s, i, j;
        interior_cell(L, t, s, i, j);
        a += F[s] * F[s];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
#pragma unroll
        for (int w = 1; w < TPB / 64; ++w) t += sh[w];
        d.red[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(64) void k_norm2(BK bk, double *out) {
    LevelDev d;
    if (!take(bk, blockIdx.x, d)) return;
    double a = 0.0;
    for (int k = threadIdx.x; k < RED_BLOCKS; k += 64) a += d.red[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
    if (threadIdx.x == 0) out[blockIdx.x] = sqrt(a / ((double)d.L.ni * d.L.nj));
}

__global__ void k_count_cycle(BK bk, int *cyc, int n) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    if (bk.act != nullptr && bk.act[c] == 0) return;
    cyc[c] = cyc[c] + 1;
}

__global__ void k_fill_int(int *p, int n, int v) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) p[c] = v;
}

// status codes (fas_status values)
constexpr int ST_OK = 0, ST_DIVERGED = -4, ST_STALLED = ST_STALLED_CODE, ST_NOT_CONVERGED = -6;

__global__ void k_batch_init(BatchCtl c, int n) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double h = c.nrm[k];
    c.h0[k] = h;
    c.hist[(size_t)k * c.hcap] = h;
    c.ndone[k] = 0;
    const bool fin = isfinite(h);
    c.stat[k] = fin ? (c.max_cycles > 0 ? ST_NOT_CONVERGED : ST_OK) : ST_DIVERGED;
    c.act[k] = (fin && c.max_cycles > 0) ? 1 : 0;
}

// after the norm of a cycle: record it, count the cycle, stop the case when
// the drop is reached, the norm is not finite or has grown beyond the limit
// (flagging the case for the roll-back of its solution), the stall test
// fails or the cap is reached
__global__ void k_batch_status(BatchCtl c, int n) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    c.rb[k] = 0;
    if (c.act[k] == 0) return;
    const double h = c.nrm[k];
    const int m = c.ndone[k] + 1;
    c.ndone[k] = m;
    c.cyc[k] = c.cyc[k] + 1;
    if (m < c.hcap) c.hist[(size_t)k * c.hcap + m] = h;
    if (!isfinite(h) || (c.growth_limit > 0.0 && h > c.growth_limit * c.h0[k])) {
        c.stat[k] = ST_DIVERGED;
        c.act[k] = 0;
        c.rb[k] = 1;
    } else if (c.drop_factor > 0.0 && h <= c.h0[k] * c.drop_factor) {
        c.stat[k] = ST_OK;
        c.act[k] = 0;
    } else if (c.stall_window > 0 && m >= c.stall_window && m < c.hcap &&
               h > c.hist[(size_t)k * c.hcap + (m - c.stall_window)] * c.stall_factor) {
        c.stat[k] = ST_STALLED;
        c.act[k] = 0;
    } else if (c.drop_factor > 0.0 && h <= c.h0[k] * c.drop_factor) {
        c.stat[k] = ST_OK;
        c.act[k] = 0;
    } else if (m >= c.max_cycles) {
        c.stat[k] = c.drop_factor > 0.0 ? ST_NOT_CONVERGED : ST_OK;
        c.act[k] = 0;
    }
}


// ------------------------------------------------- discrete Fourier analysis
// Section "Discrete Fourier Analysis": one thread per (case, pair of phase
// angles) builds the 4x4 complex Fourier symbols of the linearised JST
// operator (H_c, H_v) and of the SGS factors (L, D, U, flux splitting with
// the cutoff of eq. "cutoff" in the ARK form, eqs. "d-l-u-matrices-J",
// "d-unsteady-J", or the W form, eqs. "d-l-u-matrices-W", "d-unsteady-W"),
// forms P = (D + L) D^-1 (D + U), applies the low-storage stages of Section 4
// to the mode (U_0 = I, V_0 = P^-1 H_v, U_i = I - alpha_i dt* (P^-1 H_c
// U_{i-1} + V_{i-1}), V_i = beta_{i+1} P^-1 H_v U_i + (1 - beta_{i+1})
// V_{i-1}; G = U_s), and returns the spectral radius of G.  Per case the
// largest radius over all pairs is the amplification factor, over the pairs
// with max(|Theta_x|, |Theta_y|) >= pi/2 the smoothing factor.  Mesh and
// steps: nx cells of width 1/nx, dy = AR dx, dt* = c* dx / (|v_1| + a),
// dt = c dx / (|v_1| + a); eps2 = 0 and eps4 = (|v_k| + a) / 32 for the
// constant state.
struct cx {
    double r, i;
};
__device__ inline cx operator+(cx a, cx b) { return cx{a.r + b.r, a.i + b.i}; }
__device__ inline cx operator-(cx a, cx b) { return cx{a.r - b.r, a.i - b.i}; }
__device__ inline cx operator*(cx a, cx b) { return cx{a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ inline cx operator*(double s, cx a) { return cx{s * a.r, s * a.i}; }
__device__ inline cx conjx(cx a) { return cx{a.r, -a.i}; }
__device__ inline double norm2x(cx a) { return a.r * a.r + a.i * a.i; }
__device__ inline double cabs1(cx a) { return fabs(a.r) + fabs(a.i); }   // |Re| + |Im|, for comparisons
__device__ inline cx recipx(cx a) {
    const double q = 1.0 / norm2x(a);
    return cx{a.r * q, -a.i * q};
}
__device__ inline cx sqrtx(cx a) {
    const double m = sqrt(norm2x(a));
    if (m == 0.0) return cx{0.0, 0.0};
    const double re = sqrt(0.5 * (m + fabs(a.r)));
    if (a.r >= 0.0) return cx{re, a.i / (2.0 * re)};
    return cx{fabs(a.i) / (2.0 * re), a.i >= 0.0 ? re : -re};
}

// C = A B (4x4, row-major)
__device__ inline void cmul4(const cx *A, const cx *B, cx *C) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            cx acc = A[r * 4] * B[c];
#pragma unroll
            for (int k = 1; k < 4; ++k) acc = acc + A[r * 4 + k] * B[k * 4 + c];
            C[r * 4 + c] = acc;
        }
}

// X := A^-1 X for m right-hand columns (X row-major 4 x m), Gaussian
// elimination with partial pivoting; A is destroyed.  One reciprocal per
// pivot serves the elimination factors and the back substitution.
template <int m>
__device__ inline void csolve4(cx *A, cx *X) {
    cx ip[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        // partial pivoting: the larger of rows k and r moves to row k, for
        // each r below (static indices, so everything stays in registers)
#pragma unroll
        for (int r = k + 1; r < 4; ++r) {
            if (cabs1(A[r * 4 + k]) > cabs1(A[k * 4 + k])) {
#pragma unroll
                for (int c = 0; c < 4; ++c) { cx t = A[k * 4 + c]; A[k * 4 + c] = A[r * 4 + c]; A[r * 4 + c] = t; }
#pragma unroll
                for (int c = 0; c < m; ++c) { cx t = X[k * m + c]; X[k * m + c] = X[r * m + c]; X[r * m + c] = t; }
            }
        }
        ip[k] = recipx(A[k * 4 + k]);
#pragma unroll
        for (int r = k + 1; r < 4; ++r) {
            const cx f = A[r * 4 + k] * ip[k];
#pragma unroll
            for (int c = k + 1; c < 4; ++c) A[r * 4 + c] = A[r * 4 + c] - f * A[k * 4 + c];
#pragma unroll
            for (int c = 0; c < m; ++c) X[r * m + c] = X[r * m + c] - f * X[k * m + c];
        }
    }
#pragma unroll
    for (int k = 3; k >= 0; --k) {
#pragma unroll
        for (int c = 0; c < m; ++c) {
            cx acc = X[k * m + c];
#pragma unroll
            for (int j = k + 1; j < 4; ++j) acc = acc - A[k * 4 + j] * X[j * m + c];
            X[k * m + c] = acc * ip[k];
        }
    }
}

// X := A^-1 X for a real 4x4 A and 4 complex right-hand columns (X
// row-major), Gaussian elimination with partial pivoting; A is destroyed
__device__ inline void rsolve4(double *A, cx *X) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int r = k + 1; r < 4; ++r) {
            if (fabs(A[r * 4 + k]) > fabs(A[k * 4 + k])) {
#pragma unroll
                for (int c = 0; c < 4; ++c) { double t = A[k * 4 + c]; A[k * 4 + c] = A[r * 4 + c]; A[r * 4 + c] = t; }
#pragma unroll
                for (int c = 0; c < 4; ++c) { cx t = X[k * 4 + c]; X[k * 4 + c] = X[r * 4 + c]; X[r * 4 + c] = t; }
            }
        }
        const double ip = 1.0 / A[k * 4 + k];
#pragma unroll
        for (int r = k + 1; r < 4; ++r) {
            const double f = A[r * 4 + k] * ip;
#pragma unroll
            for (int c = k; c < 4; ++c) A[r * 4 + c] = A[r * 4 + c] - f * A[k * 4 + c];
#pragma unroll
            for (int c = 0; c < 4; ++c) X[r * 4 + c] = X[r * 4 + c] - f * X[k * 4 + c];
        }
    }
#pragma unroll
    for (int k = 3; k >= 0; --k) {
        const double ip = 1.0 / A[k * 4 + k];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            cx acc = X[k * 4 + c];
#pragma unroll
            for (int j = k + 1; j < 4; ++j) acc = acc - A[k * 4 + j] * X[j * 4 + c];
            X[k * 4 + c] = ip * acc;
        }
    }
}

// flux Jacobian dF.n/dU of the state U for the unit normal (nx, ny),
// row-major (Section 2, Euler fluxes)
__device__ inline void flux_jacobian4(const double U[4], double nx, double ny, double A[16]) {
    const double uu = U[1] / U[0], vv = U[2] / U[0];
    const double p = pres(U[0], U[1], U[2], U[3]);
    const double H = (U[3] + p) / U[0], g1 = GAM - 1.0;
    const double phi = 0.5 * g1 * (uu * uu + vv * vv), V = uu * nx + vv * ny;
    A[0] = 0.0; A[1] = nx; A[2] = ny; A[3] = 0.0;
    A[4] = phi * nx - uu * V; A[5] = V - (GAM - 2.0) * uu * nx; A[6] = uu * ny - g1 * vv * nx; A[7] = g1 * nx;
    A[8] = phi * ny - vv * V; A[9] = vv * nx - g1 * uu * ny; A[10] = V - (GAM - 2.0) * vv * ny; A[11] = g1 * ny;
    A[12] = V * (phi - H); A[13] = H * nx - g1 * uu * V; A[14] = H * ny - g1 * vv * V; A[15] = GAM * V;
}

// largest eigenvalue modulus of a 4x4 complex matrix (destroyed): the
// matrix is scaled to unit size, reduced to Hessenberg form by Householder
// reflections, then shifted QR sweeps over the whole matrix (Givens
// rotations) run until every subdiagonal entry is negligible against its
// diagonal neighbours (unit roundoff, |Re| + |Im| moduli).  Negligible
// subdiagonals are set to zero, so converged blocks decouple (their
// rotations are the identity); the Wilkinson shift comes from the lowest
// unconverged 2x2 block, with an exceptional shift on stagnation.  Every
// index is static, so the matrix stays in registers.
__device__ double spectral_radius4(cx (&H)[16]) {
    // scale to unit size: every modulus below is a plain square root
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) s = fmax(s, cabs1(H[k]));
    if (s == 0.0) return 0.0;
    const double is = 1.0 / s;
#pragma unroll
    for (int k = 0; k < 16; ++k) H[k] = is * H[k];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        double xn = 0.0;
#pragma unroll
        for (int r = k + 1; r < 4; ++r) xn += norm2x(H[r * 4 + k]);
        xn = sqrt(xn);
        const cx x0 = H[(k + 1) * 4 + k];
        const double a0 = sqrt(norm2x(x0));
        const cx ph = a0 > 0.0 ? (1.0 / a0) * x0 : cx{1.0, 0.0};
        cx v[4] = {cx{0, 0}, cx{0, 0}, cx{0, 0}, cx{0, 0}};
#pragma unroll
        for (int r = k + 1; r < 4; ++r) v[r] = H[r * 4 + k];
        v[k + 1] = x0 + xn * ph;
        double vn2 = 0.0;
#pragma unroll
        for (int r = k + 1; r < 4; ++r) vn2 += norm2x(v[r]);
        const double w = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            cx sacc = cx{0, 0};
#pragma unroll
            for (int r = k + 1; r < 4; ++r) sacc = sacc + conjx(v[r]) * H[r * 4 + c];
#pragma unroll
            for (int r = k + 1; r < 4; ++r) H[r * 4 + c] = H[r * 4 + c] - w * (v[r] * sacc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            cx sacc = cx{0, 0};
#pragma unroll
            for (int c = k + 1; c < 4; ++c) sacc = sacc + H[r * 4 + c] * v[c];
#pragma unroll
            for (int c = k + 1; c < 4; ++c) H[r * 4 + c] = H[r * 4 + c] - w * (sacc * conjx(v[c]));
        }
    }
    H[8] = H[12] = H[13] = cx{0, 0};
    for (int it = 0; it < 120; ++it) {
        bool z[4] = {true, false, false, false};
#pragma unroll
        for (int k = 1; k < 4; ++k) {
            const double sub = cabs1(H[k * 4 + k - 1]);
            z[k] = sub <= 0x1p-52 * (cabs1(H[k * 4 + k]) + cabs1(H[(k - 1) * 4 + k - 1])) || sub < 1e-300;
            if (z[k]) H[k * 4 + k - 1] = cx{0, 0};
        }
        if (z[1] && z[2] && z[3]) break;
        const int hi = !z[3] ? 3 : (!z[2] ? 2 : 1);
        cx a = H[0], b = H[1], c = H[4], d = H[5];
        if (hi == 2) { a = H[5]; b = H[6]; c = H[9]; d = H[10]; }
        if (hi == 3) { a = H[10]; b = H[11]; c = H[14]; d = H[15]; }
        cx mu;
        if (it > 0 && it % 11 == 0) {
            mu = d + cx{cabs1(c), 0.0};
        } else {
            const cx half = 0.5 * (a - d);
            const cx disc = sqrtx(half * half + b * c);
            const cx m1 = d + half + disc, m2 = d + half - disc;
            mu = norm2x(m1 - d) <= norm2x(m2 - d) ? m1 : m2;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) H[k * 5] = H[k * 5] - mu;
        double cs[3];
        cx sn[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const cx x = H[k * 4 + k], y = H[(k + 1) * 4 + k];
            const double nx = norm2x(x), ny = norm2x(y);
            double cc = 1.0;
            cx ss = cx{0, 0};
            if (ny > 0.0) {
                // c = |x| / r, s = x conj(y) / (|x| r) with r^2 = |x|^2 + |y|^2
                if (nx == 0.0) { const double iy = rsqrt(ny); cc = 0.0; ss = cx{y.r * iy, -y.i * iy}; }
                else { const double q = rsqrt(nx * (nx + ny)); cc = nx * q; ss = q * (x * conjx(y)); }
            }
            cs[k] = cc;
            sn[k] = ss;
#pragma unroll
            for (int j = k; j < 4; ++j) {
                const cx hk = H[k * 4 + j], hk1 = H[(k + 1) * 4 + j];
                H[k * 4 + j] = cc * hk + ss * hk1;
                H[(k + 1) * 4 + j] = cc * hk1 - conjx(ss) * hk;
            }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double cc = cs[k];
            const cx ss = sn[k];
#pragma unroll
            for (int i = 0; i < (k + 2 < 4 ? k + 2 : 3) + 1; ++i) {
                const cx hk = H[i * 4 + k], hk1 = H[i * 4 + k + 1];
                H[i * 4 + k] = cc * hk + conjx(ss) * hk1;
                H[i * 4 + k + 1] = cc * hk1 - ss * hk;
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) H[k * 5] = H[k * 5] + mu;
    }
    double r2 = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) r2 = fmax(r2, norm2x(H[k * 5]));
    return s * sqrt(r2);
}
__global__ __launch_bounds__(64) void k_dfa_clear(unsigned long long *amp, unsigned long long *smooth, int n) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) {
        amp[c] = 0ull;
        smooth[c] = 0ull;
    }
}

// two waves per SIMD: the register cap costs a few spills and hides more of
// the FP64 dependency latency than it loses
__global__ __launch_bounds__(64, 2) void k_dfa(const DfaCase *cases, int n_cases, long long total, double *rad,
                                            unsigned long long *amp, unsigned long long *smooth) {
    // one wave per block; every lane stays active for the reduction at the
    // end: lanes past the last pair redo the last pair and contribute nothing
    const long long tg = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = tg < total;
    const long long t = valid ? tg : total - 1;
    // case of the block's first pair by binary search over the case starts
    // (uniform across the block), then the cases that start inside it
    const long long t0 = (long long)blockIdx.x * blockDim.x;
    int lo = 0, hi = n_cases - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cases[mid].start <= t0) lo = mid;
        else hi = mid - 1;
    }
    int ci = lo;
    while (ci + 1 < n_cases && cases[ci + 1].start <= t) ++ci;
    const DfaCase P = cases[ci];
    const long long m = t - P.start;
    const int kx = (int)(m / P.ny), ky = (int)(m - (long long)kx * P.ny);
    const double tx = 2.0 * M_PI * (double)(kx - P.nx / 2 + 1) / (double)P.nx;
    const double ty = 2.0 * M_PI * (double)(ky - P.ny / 2 + 1) / (double)P.ny;
    // state, steps
    const double rho = P.u[0], v1 = P.u[1] / rho, v2 = P.u[2] / rho;
    const double a = sqrt(GAM * pres(P.u[0], P.u[1], P.u[2], P.u[3]) / rho);
    const double dx = 1.0 / (double)P.nx, dy = P.mesh ? dx / P.ar : P.ar * dx, vol = dx * dy;
    const double base = fmin(dx / (fabs(v1) + a), dy / (fabs(v2) + a));
    const double dts = P.cstar * base, dt = P.c * base;
    const cx ex = cx{cos(tx), sin(tx)}, ey = cx{cos(ty), sin(ty)};
    const cx exi = conjx(ex), eyi = conjx(ey);
    const cx dex = ex - exi, dey = ey - eyi;             // E - E^-1
    const double fx = (6.0 - 8.0 * cos(tx)) + 2.0 * cos(2.0 * tx);   // fourth difference symbols
    const double fy = (6.0 - 8.0 * cos(ty)) + 2.0 * cos(2.0 * ty);
    const double e4x = (fabs(v1) + a) / 32.0, e4y = (fabs(v2) + a) / 32.0;
    const double hv = (e4x * fx * dy + e4y * fy * dx) / vol;
    const double f = P.wform ? P.eta * dts : 1.0;
    const double diag = P.wform ? 1.0 + (P.unsteady ? 1.5 * P.eta * dts / dt : 0.0) : (P.unsteady ? 1.5 / dt : 0.0);
    // D + L, and X = D + U, then X := D^-1 (D + U) with the real D (split
    // Jacobians of the unit normals (1, 0) and (0, 1), dead afterwards);
    // P = (D + L) D^-1 (D + U) (SGS), D + L + U (exact) or I (none)
    cx Pm[16];
    if (P.precond == 2) {
#pragma unroll
        for (int k = 0; k < 16; ++k) Pm[k] = cx{k % 5 == 0 ? 1.0 : 0.0, 0.0};
    } else {
        cx DL[16], X[16];
        double Ap[16], Am[16], Bp[16], Bm[16], D[16];
        split_face(P.u, P.u, 1.0, 0.0, P.d, 0.0, 0, Ap, Am);
        split_face(P.u, P.u, 0.0, 1.0, P.d, 0.0, 0, Bp, Bm);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            D[k] = (f / vol) * (dy * (Ap[k] - Am[k]) + dx * (Bp[k] - Bm[k])) + (k % 5 == 0 ? diag : 0.0);
            const cx lk = (-(f / vol)) * (dy * Ap[k] * exi + dx * Bp[k] * eyi);
            const cx uk = (f / vol) * (dy * Am[k] * ex + dx * Bm[k] * ey);
            DL[k] = cx{D[k], 0.0} + lk;
            X[k] = cx{D[k], 0.0} + uk;
        }
        if (P.precond == 1) {
#pragma unroll
            for (int k = 0; k < 16; ++k) Pm[k] = DL[k] + (X[k] - cx{D[k], 0.0});
        } else {
            rsolve4(D, X);
            cmul4(DL, X, Pm);
        }
    }
    // H_c and H_v side by side as 8 right-hand columns, from the flux
    // Jacobians of the constant state; then [P^-1 H_c | P^-1 H_v]
    cx RHS[32];
    {
        double A[16], B[16];
        flux_jacobian4(P.u, 1.0, 0.0, A);
        flux_jacobian4(P.u, 0.0, 1.0, B);
        const double mv = -(GAM - 1.0) * (v1 * v1 + v2 * v2) / 2.0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int k = r * 4 + c;
                cx hc = (1.0 / (2.0 * vol)) * (A[k] * dy * dex + B[k] * dx * dey);
                if (P.unsteady && r == c) hc = hc + cx{1.5 / dt, 0.0};
                const double Mk = (r == 3 && c == 0) ? mv : (r == 3 && c == 3) ? GAM : (r == c ? 1.0 : 0.0);
                RHS[r * 8 + c] = hc;
                RHS[r * 8 + 4 + c] = cx{Mk * hv, 0.0};
            }
    }
    csolve4<8>(Pm, RHS);
    // the stage recursion acts on each column of G on its own (column c
    // starts from the unit vector e_c), so only one column's U and V are live
    cx G[16];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        cx u[4], v[4], w[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            u[r] = cx{r == c ? 1.0 : 0.0, 0.0};
            v[r] = RHS[r * 8 + 4 + c];
        }
        for (int st = 0; st < P.s; ++st) {
            const double al = cases[ci].alpha[st] * dts;     // from memory: no indexed register copy
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                cx acc = RHS[r * 8] * u[0];
#pragma unroll
                for (int k = 1; k < 4; ++k) acc = acc + RHS[r * 8 + k] * u[k];
                w[r] = acc;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) u[r] = cx{r == c ? 1.0 : 0.0, 0.0} - al * (w[r] + v[r]);
            if (st + 1 < P.s) {
                const double b = cases[ci].beta[st + 1];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    cx acc = RHS[r * 8 + 4] * u[0];
#pragma unroll
                    for (int k = 1; k < 4; ++k) acc = acc + RHS[r * 8 + 4 + k] * u[k];
                    w[r] = acc;
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = b * w[r] + (1.0 - b) * v[r];
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) G[r * 4 + c] = u[r];
    }
    const double r = spectral_radius4(G);
    if (rad && valid) rad[t] = r;
    const bool hf = fmax(fabs(tx), fabs(ty)) >= 0.5 * M_PI - 1e-12;
    unsigned long long ba = valid ? __builtin_bit_cast(unsigned long long, r) : 0ull;
    unsigned long long bs = hf ? ba : 0ull;
    // per-case maxima (bit patterns of non-negative doubles order like the
    // values): a wave whose lanes all belong to one case reduces over its
    // lanes first and issues one atomic per maximum
    const int c0 = __builtin_amdgcn_readfirstlane(ci);
    if (__all(ci == c0)) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long xa = __shfl_xor(ba, o), xs = __shfl_xor(bs, o);
            ba = xa > ba ? xa : ba;
            bs = xs > bs ? xs : bs;
        }
        if (threadIdx.x == 0) {
            atomicMax(&amp[c0], ba);
            if (bs) atomicMax(&smooth[c0], bs);
        }
    } else {
        if (valid) atomicMax(&amp[ci], ba);
        if (bs) atomicMax(&smooth[ci], bs);
    }
}

}  // namespace

// =================================================================== launchers
void launch_geom_interior(const Lay &L, const double *xn, const double *yn, double *geo,
                          const double *vol_children, const Lay *Lf, const double *geo_f,
                          hipStream_t st) {
    (void)vol_children;
    Lay lf = Lf ? *Lf : L;
    const double *vf = geo_f ? geo_f + (size_t)G_VOL * lf.NS : nullptr;
    hipLaunchKernelGGL(k_geom_interior, dim3(nblocks(L.NS)), dim3(TPB), 0, st, L, xn, yn, geo, vf, lf);
}

void launch_geom_ghost(const Lay &L, const double *xn, const double *yn, double *geo, hipStream_t st) {
    hipLaunchKernelGGL(k_geom_ghost, dim3(nblocks(L.NS)), dim3(TPB), 0, st, L, xn, yn, geo);
}

void launch_rotate_geometry(const Lay &L, const double *geo_ref, const double *xn, const double *yn,
                            double *geo, double c, double s, double px, double py, double omega,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_rotate_geometry, dim3(nblocks(L.NS)), dim3(TPB), 0, st, L, geo_ref, xn, yn, geo, c, s,
                       px, py, omega);
}

// one thread per padded slot of the largest case, one grid row per case
// per-cell kernels: one wave per workgroup, so that even the fine level of
// one grid (about 50k slots) spreads over every CU
constexpr int CELL_TPB = 64;
static dim3 cells_grid(const BLev &B) { return dim3(nblocks(B.max_ns, CELL_TPB), B.n); }
// one thread per cell of a rectangle (rect_cell numbering): interior cells,
// vertices, every padded cell
static dim3 interior_grid(const BLev &B) { return dim3(nblocks(B.max_ni * B.max_nj, CELL_TPB), B.n); }
static dim3 vertex_grid(const BLev &B) { return dim3(nblocks((B.max_ni + 1) * (B.max_nj + 1), CELL_TPB), B.n); }
static dim3 padded_grid(const BLev &B) {
    return dim3(nblocks((B.max_ni + 2 * NG) * (B.max_nj + 2 * NG), CELL_TPB), B.n);
}

void launch_ghost_cq(const BLev &B, int noslip, int rans, hipStream_t st) {
    hipLaunchKernelGGL(k_ghost_cq, padded_grid(B), dim3(CELL_TPB), 0, st, B.k, noslip, rans);
}

void launch_vertex_gradients(const BLev &B, hipStream_t st) {
    hipLaunchKernelGGL(k_vertex_gradients, vertex_grid(B), dim3(CELL_TPB), 0, st, B.k);
}

void launch_baldwin_lomax(const BLev &B, hipStream_t st) {
    hipLaunchKernelGGL(k_baldwin_lomax, dim3((B.max_ni + BL_COLS - 1) / BL_COLS, B.n), dim3(BL_TPB), 0, st, B.k);
}

void launch_mut_ghosts(const BLev &B, hipStream_t st) {
    hipLaunchKernelGGL(k_mut_ghosts, cells_grid(B), dim3(CELL_TPB), 0, st, B.k);
}

// Launches of at most this many cells (over all cases) take the four-lane
// residual: they leave most of the chip idle, so the flux chain's latency
// sets their time.
constexpr long long RES_QUAD_MAX_CELLS = 65536;
static long long g_four_lane_cells = RES_QUAD_MAX_CELLS;

long long four_lane_limit() { return g_four_lane_cells; }
long long set_four_lane_limit(long long cells) {
    const long long old = g_four_lane_cells;
    g_four_lane_cells = cells < 0 ? RES_QUAD_MAX_CELLS : cells;
    return old;
}

int residual_tiles(const Lay &L) { return ((L.ni + RT_I - 1) / RT_I) * ((L.nj + RT_J - 1) / RT_J); }

void launch_residual(const BLev &B, const ResArgs &a, hipStream_t st) {
    if ((long long)B.max_ni * B.max_nj * B.n <= g_four_lane_cells) {
        const dim3 grid(nblocks(4 * B.max_ni * B.max_nj, CELL_TPB), B.n);
        if (a.fp32)
            hipLaunchKernelGGL(k_residual_q<float>, grid, dim3(CELL_TPB), 0, st, B.k, a);
        else
            hipLaunchKernelGGL(k_residual_q<double>, grid, dim3(CELL_TPB), 0, st, B.k, a);
        return;
    }
    const dim3 grid = B.k.tile0 != nullptr
                          ? dim3((unsigned)B.ntiles, 1)
                          : dim3((unsigned)(((B.max_ni + RT_I - 1) / RT_I) * ((B.max_nj + RT_J - 1) / RT_J)), B.n);
    if (a.fp32)
        hipLaunchKernelGGL(k_residual_t<float>, grid, dim3(RT_TPB), 0, st, B.k, a);
    else
        hipLaunchKernelGGL(k_residual_t<double>, grid, dim3(RT_TPB), 0, st, B.k, a);
}

void launch_blocks(const BLev &B, int aw, double tau, int viscous, int fp32, hipStream_t st, int copy_u0) {
    if ((long long)B.max_ni * B.max_nj * B.n <= g_four_lane_cells) {   // the residual's small-launch rule
        const dim3 grid(nblocks(4 * B.max_ni * B.max_nj, CELL_TPB), B.n);
        if (fp32)
            hipLaunchKernelGGL(k_blocks_q<float>, grid, dim3(CELL_TPB), 0, st, B.k, aw, tau, viscous, copy_u0);
        else
            hipLaunchKernelGGL(k_blocks_q<double>, grid, dim3(CELL_TPB), 0, st, B.k, aw, tau, viscous, copy_u0);
        return;
    }
    if (fp32)
        hipLaunchKernelGGL(k_blocks<float>, interior_grid(B), dim3(CELL_TPB), 0, st, B.k, aw, tau, viscous, copy_u0);
    else
        hipLaunchKernelGGL(k_blocks<double>, interior_grid(B), dim3(CELL_TPB), 0, st, B.k, aw, tau, viscous,
                           copy_u0);
}

// Sweep configurations: four threads per row (k_sgs4 with NT threads, R
// rows per four-thread group, prefetch batches of D hyperplanes, as deep as
// the register file allows at that size and precision: FP32 rows take
// half the registers), the one-thread-per-row kernel for grids taller than
// 256 rows, the banded form of k_sgs4 (kind 5: bands of NT / 4 * R rows,
// one workgroup per band, as many bands as the tallest grid needs), and
// eight threads per row (k_sgs8: kind 8 one workgroup of NT / 8 rows per
// case, kind 9 bands of NT / 8 rows).
struct SweepCfg {
    int kind;        // 4: k_sgs4, 1: k_sgs, 5: banded k_sgs4, 8: k_sgs8, 9: banded k_sgs8
    int nt, r;
    int d64, d32;    // prefetch depth for FP64 / FP32 blocks
};
static constexpr SweepCfg SWEEP_CFGS[] = {
    {4, 64, 1, 10, 10},  {4, 128, 1, 10, 10}, {4, 256, 1, 10, 10}, {4, 512, 1, 4, 8}, {4, 1024, 1, 2, 3},
    {4, 64, 2, 5, 3},    {4, 128, 2, 5, 3},   {4, 256, 2, 5, 3},   {4, 512, 2, 2, 3}, {4, 256, 4, 2, 2},
    {1, 64, 1, 0, 0},    {1, 128, 1, 0, 0},   {1, 256, 1, 0, 0},   {1, 512, 1, 0, 0},
    {5, 64, 1, 10, 10},  {5, 128, 1, 10, 10}, {5, 256, 1, 10, 10}, {5, 128, 2, 5, 3},
    {4, 128, 1, 5, 5},   {4, 256, 1, 5, 5},   {5, 64, 1, 5, 5},    {5, 128, 1, 5, 5}, {5, 256, 1, 5, 5},
    {5, 128, 1, 3, 3},   {5, 128, 1, 4, 4},   {4, 128, 1, 3, 3},   {5, 128, 1, 2, 2},
    {5, 128, 1, 1, 1},   {5, 64, 1, 2, 2},    {5, 64, 1, 3, 3},    {4, 128, 1, 2, 2},
    {5, 64, 1, 4, 4},
    {8, 64, 1, 4, 4},    {8, 128, 1, 4, 4},   {8, 256, 1, 4, 4},   {8, 512, 1, 4, 4},
    {9, 64, 1, 4, 4},    {9, 128, 1, 4, 4},   {9, 256, 1, 4, 4},   {9, 128, 1, 3, 3},
    {9, 128, 1, 6, 6},   {9, 256, 1, 6, 6},   {9, 64, 1, 6, 6},    {8, 256, 1, 6, 6},
    {5, 64, 2, 2, 2},    {5, 64, 2, 3, 3},
};
constexpr int N_SWEEP_CFGS = (int)(sizeof(SWEEP_CFGS) / sizeof(SWEEP_CFGS[0]));

int sweep_cfg_count() { return N_SWEEP_CFGS; }

static int cfg_group_rows(int cfg) {
    const SweepCfg &c = SWEEP_CFGS[cfg];
    return c.kind == 1 ? c.nt : (c.kind == 8 || c.kind == 9) ? c.nt / 8 : c.nt / 4 * c.r;
}

bool sweep_cfg_banded(int cfg) { return SWEEP_CFGS[cfg].kind == 5 || SWEEP_CFGS[cfg].kind == 9; }

int sweep_cfg_bands(int cfg, int max_nj) {
    const int nr = cfg_group_rows(cfg);
    return sweep_cfg_banded(cfg) ? (max_nj + nr - 1) / nr : 1;
}

int sweep_cfg_rows(int cfg, int max_nj) { return cfg_group_rows(cfg) * sweep_cfg_bands(cfg, max_nj); }

void sweep_cfg_info(int cfg, int *kind, int *threads, int *rows, int *d64, int *d32) {
    const SweepCfg &c = SWEEP_CFGS[cfg];
    *kind = c.kind == 4 ? 0 : c.kind == 1 ? 1 : c.kind == 5 ? 2 : c.kind == 8 ? 3 : 4;
    *threads = c.nt;
    *rows = cfg_group_rows(cfg);
    *d64 = c.d64;
    *d32 = c.d32;
}

// one workgroup per case, by height (also the fall-back of a banded launch
// whose workgroups cannot all be resident)
int sweep_cfg_plain(int max_nj) {
    if (max_nj <= 16) return 0;
    if (max_nj <= 32) return 25;
    if (max_nj <= 64) return 19;
    if (max_nj <= 128) return 3;
    if (max_nj <= 256) return 4;
    return 13;
}

// Default by height and precision, from timings of every configuration on
// the three levels of a 256 x 128 grid: one 128-thread workgroup with
// prefetch depth 3 up to 32 rows; above, bands of 16 rows (one wave each,
// no workgroup barrier) with depth 4 for FP64 blocks and depth 5 for FP32
// blocks (a FP32 block row is one 16-byte load instead of two, so the same
// depth keeps fewer loads in flight).
int sweep_cfg_default(int max_nj, int fp32) {
    if (max_nj <= 32) return sweep_cfg_plain(max_nj);
    return fp32 ? 20 : 31;
}
// Banded launches wait on neighbouring workgroups: they are used only when
// the whole grid can be resident at once.
template <typename K>
static int resident_blocks(K kernel, int nt, size_t shm) {
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void *>(kernel), nt, shm) !=
            hipSuccess)
        return 0;
    return per * ncu;
}

template <typename T> static void sgs_dispatch(const BLev &B, const SweepArgs &a0, hipStream_t st);

// one configuration of the table, instantiated at compile time; a banded
// launch whose workgroups cannot all be resident falls back to one
// workgroup per case
template <typename T, int C>
static void sgs_launch_cfg(const BLev &B, const SweepArgs &a0, hipStream_t st) {
    constexpr SweepCfg c = SWEEP_CFGS[C];
    constexpr int D = sizeof(T) == 4 ? c.d32 : c.d64;
    const int nwl = B.max_nw > 0 ? B.max_nw : 1;
    const size_t shm = (size_t)nwl * 4 * sizeof(T);
    const size_t shm4 = (size_t)nwl * 20 * sizeof(T);
    SweepArgs a = a0;
    a.bands = sweep_cfg_bands(C, B.max_nj);
    auto banded = [&](auto kernel) {
        if (B.n * a.bands <= resident_blocks(kernel, c.nt, shm4)) {
            hipLaunchKernelGGL(kernel, dim3(B.n * a.bands), dim3(c.nt), shm4, st, B.k, a);
        } else {
            BLev B1 = B;
            B1.sweep_cfg = sweep_cfg_plain(B.max_nj);
            sgs_dispatch<T>(B1, a0, st);
        }
    };
    if constexpr (c.kind == 1) {
        hipLaunchKernelGGL((k_sgs<T, c.nt>), dim3(B.n), dim3(c.nt), shm, st, B.k, a);
    } else if constexpr (c.kind == 4) {
        hipLaunchKernelGGL((k_sgs4<T, c.nt, c.r, D, false>), dim3(B.n), dim3(c.nt), shm4, st, B.k, a);
    } else if constexpr (c.kind == 5) {
        banded(k_sgs4<T, c.nt, c.r, D, true>);
    } else if constexpr (c.kind == 8) {
        hipLaunchKernelGGL((k_sgs8<T, c.nt / 64, D, false>), dim3(B.n), dim3(c.nt), shm4, st, B.k, a);
    } else {
        static_assert(c.kind == 9, "unknown sweep kind");
        banded(k_sgs8<T, c.nt / 64, D, true>);
    }
}

template <typename T, int... Cs>
static void sgs_select(int cfg, const BLev &B, const SweepArgs &a0, hipStream_t st,
                       std::integer_sequence<int, Cs...>) {
    ((cfg == Cs ? (sgs_launch_cfg<T, Cs>(B, a0, st), 0) : 0), ...);
}

template <typename T>
static void sgs_dispatch(const BLev &B, const SweepArgs &a0, hipStream_t st) {
    constexpr int FP32 = sizeof(T) == 4 ? 1 : 0;
    int cfg = B.sweep_cfg >= 0 ? B.sweep_cfg : sweep_cfg_default(B.max_nj, FP32);
    if (cfg >= N_SWEEP_CFGS || sweep_cfg_rows(cfg, B.max_nj) < B.max_nj) cfg = sweep_cfg_default(B.max_nj, FP32);
    sgs_select<T>(cfg, B, a0, st, std::make_integer_sequence<int, N_SWEEP_CFGS>());
}

void launch_sgs(const BLev &B, const SweepArgs &a, int fp32, hipStream_t st) {
    if (fp32) sgs_dispatch<float>(B, a, st);
    else sgs_dispatch<double>(B, a, st);
}

void launch_dinv(const BLev &B, int fp32, hipStream_t st) {
    if (fp32)
        hipLaunchKernelGGL(k_dinv<float>, cells_grid(B), dim3(CELL_TPB), 0, st, B.k);
    else
        hipLaunchKernelGGL(k_dinv<double>, cells_grid(B), dim3(CELL_TPB), 0, st, B.k);
}

void launch_restrict(const BLev &Bf, const BLev &Bc, int fin, int fout, int fout2, hipStream_t st) {
    const RJob j = {fin, 1.0, FLD_NONE, 0.0, fout, fout2};
    launch_restrict_jobs(Bf, Bc, &j, 1, 0, st);
}

void launch_restrict_jobs(const BLev &Bf, const BLev &Bc, const RJob *jobs, int njobs, int mut, hipStream_t st) {
    hipLaunchKernelGGL(k_restrict, cells_grid(Bc), dim3(CELL_TPB), 0, st, Bf.k, Bc.k, jobs[0],
                       njobs > 1 ? jobs[1] : jobs[0], njobs > 1 ? 2 : 1, mut);
}

void launch_prolong(const BLev &Bf, const BLev &Bc, hipStream_t st) {
    hipLaunchKernelGGL(k_prolong, cells_grid(Bf), dim3(CELL_TPB), 0, st, Bf.k, Bc.k);
}

void launch_save_u(const BLev &B, hipStream_t st) {
    hipLaunchKernelGGL(k_axpby, cells_grid(B), dim3(CELL_TPB), 0, st, B.k, 1.0, (int)FLD_U, 0.0, (int)FLD_NONE,
                       (int)FLD_ULAST);
}

void launch_rollback(const BLev &B, const int *rb, hipStream_t st) {
    hipLaunchKernelGGL(k_rollback, cells_grid(B), dim3(CELL_TPB), 0, st, B.k, rb);
}

void launch_axpby(const BLev &B, double a, int fx, double b, int fy, int fout, hipStream_t st) {
    hipLaunchKernelGGL(k_axpby, cells_grid(B), dim3(CELL_TPB), 0, st, B.k, a, fx, b, fy, fout);
}

void launch_pack(const Lay &L, const double *padded, double *natural, int ncomp, hipStream_t st) {
    hipLaunchKernelGGL(k_pack, dim3(nblocks(L.ni * L.nj)), dim3(TPB), 0, st, L, padded, natural, ncomp);
}

void launch_unpack(const Lay &L, const double *natural, double *padded, int ncomp, hipStream_t st) {
    hipLaunchKernelGGL(k_unpack, dim3(nblocks(L.ni * L.nj)), dim3(TPB), 0, st, L, natural, padded, ncomp);
}

int norm_scratch_size() { return RED_BLOCKS; }

void launch_norm(const BLev &B, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_norm1, dim3(RED_BLOCKS, B.n), dim3(TPB), 0, st, B.k);
    hipLaunchKernelGGL(k_norm2, dim3(B.n), dim3(64), 0, st, B.k, out);
}

void launch_count_cycle(const BLev &B, int *cyc, hipStream_t st) {
    hipLaunchKernelGGL(k_count_cycle, dim3(nblocks(B.n, 64)), dim3(64), 0, st, B.k, cyc, B.n);
}

void launch_fill_int(int *p, int n, int v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_int, dim3(nblocks(n, 64)), dim3(64), 0, st, p, n, v);
}

void launch_batch_init(const BatchCtl &c, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_init, dim3(nblocks(n, 64)), dim3(64), 0, st, c, n);
}

void launch_batch_status(const BatchCtl &c, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_status, dim3(nblocks(n, 64)), dim3(64), 0, st, c, n);
}

// Non-negative doubles order like their bit patterns as unsigned integers,
// so the per-case maxima are reduced with an integer atomic maximum.
void launch_dfa(const DfaCase *d_cases, int n_cases, long long total, double *rad, double *amp, double *smooth,
                hipStream_t st) {
    unsigned long long *ua = reinterpret_cast<unsigned long long *>(amp);
    unsigned long long *us = reinterpret_cast<unsigned long long *>(smooth);
    hipLaunchKernelGGL(k_dfa_clear, dim3(nblocks(n_cases, 64)), dim3(64), 0, st, ua, us, n_cases);
    if (total > 0)
        hipLaunchKernelGGL(k_dfa, dim3((unsigned)((total + 63) / 64)), dim3(64), 0, st, d_cases, n_cases, total, rad,
                           ua, us);
}

}  // namespace fas
