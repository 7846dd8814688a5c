// HIP kernels (gfx950) of the discrete adjoint of the steady fine-level
// residual: vector-Jacobian products, parameter derivatives, the wall
// force and its gradient, and the transposed SGS preconditioner.
//
// Derivatives are exact derivatives of the discrete residual (Section 2:
// JST flux, viscous flux, boundary conditions), taken by forward-mode dual
// numbers on a cell's local stencil, with the eddy viscosity frozen at the
// state.  Layout: fas_internal.h.
#include "fas_internal.h"
#include "fas_geom.h"
#include "fas_cells.h"

#include <cmath>

namespace fas {

namespace {

constexpr int TPB = 256;
constexpr double SUTH = 110.4 / 288.15;
inline int nblocks(int n, int t = TPB) { return (n + t - 1) / t; }

// ------------------------------------------------------------- dual numbers
// value and four derivative lanes
struct D4 {
    double v, d[4];
};

__device__ inline D4 dc(double v) { return D4{v, {0.0, 0.0, 0.0, 0.0}}; }
__device__ inline D4 operator+(const D4 &a, const D4 &b) {
    return D4{a.v + b.v, {a.d[0] + b.d[0], a.d[1] + b.d[1], a.d[2] + b.d[2], a.d[3] + b.d[3]}};
}
__device__ inline D4 operator-(const D4 &a, const D4 &b) {
    return D4{a.v - b.v, {a.d[0] - b.d[0], a.d[1] - b.d[1], a.d[2] - b.d[2], a.d[3] - b.d[3]}};
}
__device__ inline D4 operator-(const D4 &a) { return D4{-a.v, {-a.d[0], -a.d[1], -a.d[2], -a.d[3]}}; }
__device__ inline D4 operator*(const D4 &a, const D4 &b) {
    D4 r;
    r.v = a.v * b.v;
#pragma unroll
    for (int k = 0; k < 4; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
__device__ inline D4 operator/(const D4 &a, const D4 &b) {
    D4 r;
    r.v = a.v / b.v;
    const double ib = 1.0 / b.v;
#pragma unroll
    for (int k = 0; k < 4; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
    return r;
}
__device__ inline D4 operator*(double s, const D4 &a) {
    return D4{s * a.v, {s * a.d[0], s * a.d[1], s * a.d[2], s * a.d[3]}};
}
__device__ inline D4 operator*(const D4 &a, double s) { return s * a; }
__device__ inline D4 operator+(const D4 &a, double s) { return D4{a.v + s, {a.d[0], a.d[1], a.d[2], a.d[3]}}; }
__device__ inline D4 operator+(double s, const D4 &a) { return a + s; }
__device__ inline D4 operator-(const D4 &a, double s) { return D4{a.v - s, {a.d[0], a.d[1], a.d[2], a.d[3]}}; }
__device__ inline D4 operator-(double s, const D4 &a) { return dc(s) - a; }
__device__ inline D4 operator/(const D4 &a, double s) { return a * (1.0 / s); }
__device__ inline D4 chain(const D4 &a, double f, double df) {
    return D4{f, {df * a.d[0], df * a.d[1], df * a.d[2], df * a.d[3]}};
}
__device__ inline D4 dsqrt(const D4 &a) {
    const double r = sqrt(a.v);
    return chain(a, r, 0.5 / r);
}
__device__ inline D4 dcbrt(const D4 &a) {
    const double r = cbrt(a.v);
    return chain(a, r, 1.0 / (3.0 * r * r));
}
__device__ inline D4 dpow(const D4 &a, double e) {
    const double r = pow(a.v, e);
    return chain(a, r, e * pow(a.v, e - 1.0));
}
__device__ inline D4 dabs(const D4 &a) { return a.v < 0.0 ? -a : a; }
__device__ inline D4 dmax(const D4 &a, const D4 &b) { return (b.v > a.v) ? b : a; }
__device__ inline D4 dmin(const D4 &a, const D4 &b) { return (b.v < a.v) ? b : a; }

// --------------------------------------------------------------- geometry
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

// --------------------------------------------- local residual, dual numbers
// Everything a cell's residual needs is rebuilt from the interior states of
// its stencil: ghost states through the boundary conditions, pressure,
// sensor and spectral radii, vertex gradients.  Interior cell (si, sj)
// carries the derivative seed (lane k = d/du_k of that cell); the far-field
// state may carry parameter lanes instead.
struct Ctx {
    Lay L;
    const double *geo, *u, *mut;
    D4 uinf[4];
    D4 mu_inf;
    double pr, prt, kappa2c;
    int rans, noslip, fine, viscous;
    int part;             // 0: F = f^c + f^v; 1: f^c alone; 2: f^v alone (Section 4.1 split)
    int inv;              // 0: the face flux's inviscid part is left out (its derivative is zero)
    int si, sj;
    int gp[4], gs[4];     // geometry seeds: plane and slot of derivative lane k (-1: none)
};

using ::fas::gsqrt;
__device__ inline D4 gsqrt(const D4 &a) { return dsqrt(a); }

// a metric value: plain, or as a dual number seeded on the geometry lanes
template <class G> struct GeoRead;
template <> struct GeoRead<double> {
    __device__ static double at(const Ctx &c, int p, int s) { return c.geo[p * c.L.NS + s]; }
};
template <> struct GeoRead<D4> {
    __device__ static D4 at(const Ctx &c, int p, int s) {
        D4 v = dc(c.geo[p * c.L.NS + s]);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (c.gp[k] == p && c.gs[k] == s) v.d[k] = 1.0;
        return v;
    }
};
template <class G>
__device__ inline G gget(const Ctx &c, int p, int s) {
    return GeoRead<G>::at(c, p, s);
}

__device__ inline void cell_u(const Ctx &c, int i, int j, D4 o[4]) {
    const int s = c.L.slot(i, j), NS = c.L.NS;
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = dc(c.u[k * NS + s]);
    if (i == c.si && j == c.sj) {
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k].d[k] = 1.0;
    }
}

__device__ inline D4 dpres(const D4 U[4]) {
    return (GAM - 1.0) * (U[3] - 0.5 * (U[1] * U[1] + U[2] * U[2]) / U[0]);
}

template <class G>
__device__ inline void unit(G sx, G sy, G &nx, G &ny) {
    G ln = gsqrt(sx * sx + sy * sy);
    nx = sx / ln;
    ny = sy / ln;
}

// Riemann-invariant far-field state (Section 2)
template <class G>
__device__ void farfield(const D4 ui[4], const D4 uf[4], G nx, G ny, D4 out[4]) {
    const double g1 = GAM - 1.0;
    D4 rho = ui[0];
    D4 vx = ui[1] / rho, vy = ui[2] / rho;
    D4 p = dpres(ui);
    D4 a = dsqrt(GAM * p / rho);
    D4 rinf = uf[0];
    D4 vxf = uf[1] / rinf, vyf = uf[2] / rinf;
    D4 pf = dpres(uf);
    D4 af = dsqrt(GAM * pf / rinf);
    D4 vn = vx * nx + vy * ny;
    D4 vnf = vxf * nx + vyf * ny;
    D4 rp = vn + 2.0 * a / g1;
    D4 rm = vnf - 2.0 * af / g1;
    D4 vnb = 0.5 * (rp + rm);
    D4 ab = 0.25 * g1 * (rp - rm);
    const bool outf = vnb.v > 0.0;
    D4 sent = outf ? p / dpow(rho, GAM) : pf / dpow(rinf, GAM);
    D4 tx = outf ? vx - vn * nx : vxf - vnf * nx;
    D4 ty = outf ? vy - vn * ny : vyf - vnf * ny;
    D4 base = ab * ab / (GAM * sent);
    D4 rhob = base * base * dsqrt(base);
    D4 pb = rhob * ab * ab / GAM;
    D4 ub = tx + vnb * nx, vb = ty + vnb * ny;
    out[0] = rhob;
    out[1] = rhob * ub;
    out[2] = rhob * vb;
    out[3] = pb / g1 + 0.5 * rhob * (ub * ub + vb * vb);
}

// state of (i, j): i interior, j in [-2, nj + 2)
template <class G>
__device__ void jrow(const Ctx &c, int i, int j, D4 o[4]) {
    const Lay &L = c.L;
    const int NS = L.NS;
    if (j >= 0 && j < L.nj) {
        cell_u(c, i, j, o);
        return;
    }
    if (j < 0) {
        const int k = -1 - j;
        if (cut_col(L, i)) {
            cell_u(c, L.ni - 1 - i, k, o);
            return;
        }
        D4 ui[4];
        cell_u(c, i, k, ui);
        if (c.noslip) {
            o[0] = ui[0];
            o[1] = -ui[1];
            o[2] = -ui[2];
            o[3] = ui[3];
        } else {
            const int f = L.slot(i, 0);
            G nx, ny;
            unit<G>(gget<G>(c, G_SETA_X, f), gget<G>(c, G_SETA_Y, f), nx, ny);
            D4 mn = ui[1] * nx + ui[2] * ny;
            o[0] = ui[0];
            o[1] = ui[1] - 2.0 * mn * nx;
            o[2] = ui[2] - 2.0 * mn * ny;
            o[3] = ui[3];
        }
        return;
    }
    const int k = j - L.nj;
    D4 ui[4];
    cell_u(c, i, L.nj - 1 - k, ui);
    const int f = L.slot(i, L.nj);
    G nx, ny;
    unit<G>(gget<G>(c, G_SETA_X, f), gget<G>(c, G_SETA_Y, f), nx, ny);
    farfield<G>(ui, c.uinf, nx, ny, o);
}

// state of any padded cell (i, j), i and j in [-2, n + 2)
template <class G>
__device__ void state(const Ctx &c, int i, int j, D4 o[4]) {
    const Lay &L = c.L;
    if (i >= 0 && i < L.ni) {
        jrow<G>(c, i, j, o);
        return;
    }
    const int jc = min(max(j, 0), L.nj - 1);
    D4 src[4];
    G nx, ny;
    if (i < 0) {
        jrow<G>(c, -1 - i, j, src);
        const int f = L.slot(0, jc);
        unit<G>(-gget<G>(c, G_SXI_X, f), -gget<G>(c, G_SXI_Y, f), nx, ny);
    } else {
        jrow<G>(c, L.ni - 1 - (i - L.ni), j, src);
        const int f = L.slot(L.ni, jc);
        unit<G>(gget<G>(c, G_SXI_X, f), gget<G>(c, G_SXI_Y, f), nx, ny);
    }
    farfield<G>(src, c.uinf, nx, ny, o);
}

// interior cell whose state a padded cell's state is built from
__device__ void source_of(const Lay &L, int i, int j, int &si, int &sj) {
    if (i < 0) i = -1 - i;
    else if (i >= L.ni) i = L.ni - 1 - (i - L.ni);
    if (j >= 0 && j < L.nj) {
        si = i;
        sj = j;
    } else if (j < 0) {
        const int k = -1 - j;
        si = cut_col(L, i) ? L.ni - 1 - i : i;
        sj = k;
    } else {
        si = i;
        sj = L.nj - 1 - (j - L.nj);
    }
}

struct CQ {
    D4 U[4], p, q, rxi, reta, T;
};

// Section 2: pressure, sensor quantity, corrected spectral radii, p / rho
template <class G>
__device__ void cell_q(const Ctx &c, int i, int j, CQ &o) {
    state<G>(c, i, j, o.U);
    const int s = c.L.slot(i, j);
    const D4 &r = o.U[0];
    D4 vx = o.U[1] / r, vy = o.U[2] / r;
    o.p = dpres(o.U);
    D4 a = dsqrt(GAM * o.p / r);
    o.q = c.rans ? o.p / dpow(r, GAM) : o.p;
    const G sb0 = gget<G>(c, G_SB0, s), sb1 = gget<G>(c, G_SB1, s);
    const G sb2 = gget<G>(c, G_SB2, s), sb3 = gget<G>(c, G_SB3, s);
    D4 rxi = dabs(vx * sb0 + vy * sb1) + a * gsqrt(sb0 * sb0 + sb1 * sb1);
    D4 reta = dabs(vx * sb2 + vy * sb3) + a * gsqrt(sb2 * sb2 + sb3 * sb3);
    D4 t = reta / rxi;
    o.rxi = rxi * (1.0 + dcbrt(t * t));
    t = rxi / reta;
    o.reta = reta * (1.0 + dcbrt(t * t));
    o.T = o.p / r;
}

// Green-Gauss gradients of (u, v, T) at vertex (I, J) over the four cell
// centres SW, SE, NE, NW
template <class G>
__device__ void vertex_grad(const Ctx &c, int I, int J, D4 g[6]) {
    const int ci[4] = {I - 1, I, I, I - 1}, cj[4] = {J - 1, J - 1, J, J};
    G X[4], Y[4];
    D4 U[4], V[4], T[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int s = c.L.slot(ci[k], cj[k]);
        X[k] = gget<G>(c, G_XC, s);
        Y[k] = gget<G>(c, G_YC, s);
        D4 st[4];
        state<G>(c, ci[k], cj[k], st);
        U[k] = st[1] / st[0];
        V[k] = st[2] / st[0];
        T[k] = dpres(st) / st[0];
    }
    const G A = 0.5 * ((X[2] - X[0]) * (Y[3] - Y[1]) - (Y[2] - Y[0]) * (X[3] - X[1]));
    const D4 *phi[3] = {U, V, T};
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        D4 gx = dc(0.0), gy = dc(0.0);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int a = e, b = (e + 1) & 3;
            D4 m = 0.5 * (phi[f][a] + phi[f][b]);
            D4 tx = m * (Y[b] - Y[a]);
            D4 ty = m * (X[a] - X[b]);
            if (e == 0) {
                gx = tx;
                gy = ty;
            } else {
                gx = gx + tx;
                gy = gy + ty;
            }
        }
        g[2 * f] = gx / A;
        g[2 * f + 1] = gy / A;
    }
}

__device__ inline D4 dsutherland(const D4 &T, const D4 &mu_inf) {
    return ((mu_inf * (T * dsqrt(T))) * (1.0 + SUTH)) / (T + SUTH);
}

// JST face flux (central C, dissipation / viscous V) between L and R with
// outer neighbours LL and RR (Section 2), as in the primal residual
template <class G>
__device__ void face(const Ctx &c, int iL, int jL, int iR, int jR, int iLL, int jLL, int iRR, int jRR,
                     bool xi_face, G sx, G sy, bool wall, int vAi, int vAj, int vBi, int vBj,
                     D4 C[4], D4 V[4]) {
    CQ L, R;
    cell_q<G>(c, iL, jL, L);
    cell_q<G>(c, iR, jR, R);
    if (!c.inv) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            C[k] = dc(0.0);
            V[k] = dc(0.0);
        }
    } else if (wall) {
        D4 pw = 0.5 * (L.p + R.p);
        C[0] = dc(0.0);
        C[1] = pw * sx;
        C[2] = pw * sy;
        C[3] = dc(0.0);
#pragma unroll
        for (int k = 0; k < 4; ++k) V[k] = dc(0.0);
    } else {
        D4 qsL = L.U[1] * sx + L.U[2] * sy, vsL = qsL / L.U[0];
        D4 qsR = R.U[1] * sx + R.U[2] * sy, vsR = qsR / R.U[0];
        D4 FL[4] = {qsL, L.U[1] * vsL + L.p * sx, L.U[2] * vsL + L.p * sy, (L.U[3] + L.p) * vsL};
        D4 FR[4] = {qsR, R.U[1] * vsR + R.p * sx, R.U[2] * vsR + R.p * sy, (R.U[3] + R.p) * vsR};
#pragma unroll
        for (int k = 0; k < 4; ++k) C[k] = 0.5 * (FL[k] + FR[k]);
        D4 rf = xi_face ? dmax(L.rxi, R.rxi) : dmax(L.reta, R.reta);
        D4 wL[4] = {L.U[0], L.U[1], L.U[2], L.U[3] + L.p};
        D4 wR[4] = {R.U[0], R.U[1], R.U[2], R.U[3] + R.p};
        D4 d[4];
        if (c.fine) {
            CQ LL, RR;
            cell_q<G>(c, iLL, jLL, LL);
            cell_q<G>(c, iRR, jRR, RR);
            D4 sLs = dabs(((R.q - 2.0 * L.q) + LL.q) / (((R.q + 2.0 * L.q) + LL.q) + 0.001));
            D4 sRs = dabs(((RR.q - 2.0 * R.q) + L.q) / (((RR.q + 2.0 * R.q) + L.q) + 0.001));
            D4 sf = dmin(dc(0.25), dmax(sLs, sRs));
            D4 e2 = sf * rf;
            D4 e4 = dmax(dc(0.0), rf / 32.0 - 2.0 * e2);
            D4 wLL[4] = {LL.U[0], LL.U[1], LL.U[2], LL.U[3] + LL.p};
            D4 wRR[4] = {RR.U[0], RR.U[1], RR.U[2], RR.U[3] + RR.p};
#pragma unroll
            for (int k = 0; k < 4; ++k)
                d[k] = e2 * (wR[k] - wL[k]) - e4 * (((wRR[k] - 3.0 * wR[k]) + 3.0 * wL[k]) - wLL[k]);
        } else {
            D4 e2 = c.kappa2c * rf;
#pragma unroll
            for (int k = 0; k < 4; ++k) d[k] = e2 * (wR[k] - wL[k]);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) V[k] = -d[k];
    }
    if (c.viscous) {
        D4 gA[6], gB[6];
        vertex_grad<G>(c, vAi, vAj, gA);
        vertex_grad<G>(c, vBi, vBj, gB);
        D4 fux = 0.5 * (gA[0] + gB[0]), fuy = 0.5 * (gA[1] + gB[1]);
        D4 fwx = 0.5 * (gA[2] + gB[2]), fwy = 0.5 * (gA[3] + gB[3]);
        D4 fTx = 0.5 * (gA[4] + gB[4]), fTy = 0.5 * (gA[5] + gB[5]);
        D4 fvx = 0.5 * (L.U[1] / L.U[0] + R.U[1] / R.U[0]);
        D4 fvy = 0.5 * (L.U[2] / L.U[0] + R.U[2] / R.U[0]);
        D4 fT = 0.5 * (L.T + R.T);
        D4 mu = dsutherland(fT, c.mu_inf);
        const int sL = c.L.slot(iL, jL), sR = c.L.slot(iR, jR);
        const double mt = 0.5 * (c.mut[sL] + c.mut[sR]);
        D4 mue = mu + mt;
        D4 kc = (mu / c.pr + mt / c.prt) * (GAM / (GAM - 1.0));
        D4 div = fux + fwy;
        D4 txx = mue * (2.0 * fux - (2.0 / 3.0) * div);
        D4 tyy = mue * (2.0 * fwy - (2.0 / 3.0) * div);
        D4 txy = mue * (fuy + fwx);
        D4 qx = kc * fTx, qy = kc * fTy;
        D4 G1 = txx * sx + txy * sy;
        D4 G2 = txy * sx + tyy * sy;
        D4 G3 = ((fvx * txx + fvy * txy) + qx) * sx + ((fvx * txy + fvy * tyy) + qy) * sy;
        V[1] = V[1] - G1;
        V[2] = V[2] - G2;
        V[3] = V[3] - G3;
    }
}

// F of interior cell (i, j) per unit volume (steady, no forcing)
template <class G>
__device__ void cell_residual(const Ctx &c, int i, int j, D4 F[4]) {
    const Lay &L = c.L;
    const int s = L.slot(i, j), NJ = L.NJ;
    D4 wC[4], wV[4], eC[4], eV[4], sC[4], sV[4], nC[4], nV[4];
    face<G>(c, i - 1, j, i, j, i - 2, j, i + 1, j, true, gget<G>(c, G_SXI_X, s), gget<G>(c, G_SXI_Y, s), false,
            i, j, i, j + 1, wC, wV);
    face<G>(c, i, j, i + 1, j, i - 1, j, i + 2, j, true, gget<G>(c, G_SXI_X, s + NJ),
            gget<G>(c, G_SXI_Y, s + NJ), false, i + 1, j, i + 1, j + 1, eC, eV);
    const bool wall = (j == 0) && !cut_col(L, i);
    face<G>(c, i, j - 1, i, j, i, j - 2, i, j + 1, false, gget<G>(c, G_SETA_X, s), gget<G>(c, G_SETA_Y, s),
            wall, i, j, i + 1, j, sC, sV);
    face<G>(c, i, j, i, j + 1, i, j - 1, i, j + 2, false, gget<G>(c, G_SETA_X, s + NJ + 1),
            gget<G>(c, G_SETA_Y, s + NJ + 1), false, i, j + 1, i + 1, j + 1, nC, nV);
    const G vol = gget<G>(c, G_VOL, s);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        D4 fc = (eC[k] - wC[k]) + (nC[k] - sC[k]);
        D4 fv = (eV[k] - wV[k]) + (nV[k] - sV[k]);
        if (c.part == 0) F[k] = fc / vol + fv / vol;
        else if (c.part == 1) F[k] = fc / vol;
        else F[k] = fv / vol;
    }
}

__device__ void make_ctx(Ctx &c, const Lay &L, const double *geo, const double *u, const double *mut,
                         const Phys &ph) {
    c.L = L;
    c.geo = geo;
    c.u = u;
    c.mut = mut;
#pragma unroll
    for (int k = 0; k < 4; ++k) c.uinf[k] = dc(ph.uinf[k]);
    c.mu_inf = dc(ph.mu_inf);
    c.pr = ph.pr;
    c.prt = ph.prt;
    c.kappa2c = ph.kappa2c;
    c.rans = ph.rans;
    c.noslip = ph.rans;
    c.fine = 1;
    c.viscous = ph.rans;
    c.part = 0;
    c.inv = 1;
    c.si = c.sj = -1000000;
#pragma unroll
    for (int k = 0; k < 4; ++k) c.gp[k] = c.gs[k] = -1;
}

// ------------------------------------------------------------------ kernels
// out += (dF/du)^T lam, face by face.  F_c is the sum of c's four face
// fluxes (east and north added, west and south subtracted) over vol_c, and
// an interior face's flux is the same value for both of its cells, so
//     (dF/du)^T lam = sum over faces f of (dflux_f/du)^T mu_f,
//     mu_f = lam_L / vol_L - lam_R / vol_R
// (a side that is not an interior cell drops out: boundary faces belong to
// their one interior cell; on the wake cut each row-0 cell keeps its own
// south face, as in the residual).  A face's flux depends on the states of
// its JST line (LL, L, R, RR) and, for viscous faces, of the four cells
// around each of its two vertices: at most 8 cells, each mapped through the
// boundary conditions to the interior cell its state comes from.  Thread
// (face, q) seeds the q-th distinct such source cell, evaluates the flux
// with dual numbers, and scatters the four products to that cell.  part
// selects F, its convective part f^c or its dissipative and viscous part
// f^v.  out must be zeroed first.
constexpr int VJP_SOURCES = 8;

__global__ __launch_bounds__(TPB) void k_vjp(Lay L, const double *geo, const double *u, const double *mut,
                                             Phys ph, const double *lam, double *out, int part) {
    const int q = blockIdx.y;
    const int t = blockIdx.x * TPB + threadIdx.x;
    const int nif = (L.ni + 1) * L.nj;
    int sf, a, b;
    bool xi = t < nif;
    if (xi) rect_cell(L, t, L.ni + 1, L.nj, 0, sf, a, b);                 // face between (a - 1, b) and (a, b)
    else if (!rect_cell(L, t - nif, L.ni, L.nj + 1, 0, sf, a, b)) return;  // face between (a, b - 1) and (a, b)
    const int iL = xi ? a - 1 : a, jL = xi ? b : b - 1;
    const int iLL = xi ? a - 2 : a, jLL = xi ? b : b - 2, iRR = xi ? a + 1 : a, jRR = xi ? b : b + 1;
    const int vAi = a, vAj = b, vBi = xi ? a : a + 1, vBj = xi ? b + 1 : b;
    // stencil: the JST line, then the remaining cells around the vertices
    int pi[VJP_SOURCES] = {iLL, iL, a, iRR, 0, 0, 0, 0}, pj[VJP_SOURCES] = {jLL, jL, b, jRR, 0, 0, 0, 0};
    if (xi) {
        pi[4] = a - 1; pj[4] = b - 1; pi[5] = a; pj[5] = b - 1;
        pi[6] = a - 1; pj[6] = b + 1; pi[7] = a; pj[7] = b + 1;
    } else {
        pi[4] = a - 1; pj[4] = b - 1; pi[5] = a - 1; pj[5] = b;
        pi[6] = a + 1; pj[6] = b - 1; pi[7] = a + 1; pj[7] = b;
    }
    const int np = ph.rans ? 8 : 4;
    int si = 0, sj = 0, n = 0;
    for (int p = 0; p < np; ++p) {
        int ci, cj;
        source_of(L, pi[p], pj[p], ci, cj);
        bool dup = false;
        for (int r = 0; r < p; ++r) {
            int di, dj;
            source_of(L, pi[r], pj[r], di, dj);
            dup = dup || (di == ci && dj == cj);
        }
        if (!dup) {
            if (n == q) {
                si = ci;
                sj = cj;
            }
            ++n;
        }
    }
    if (q >= n) return;
    // The inviscid part depends on the JST line (positions 0-3) only, the
    // viscous part on L, R and the vertex cells (positions 1, 2, 4-7): a part
    // whose cells do not include the seeded source has a zero derivative and
    // is not evaluated.
    bool dep_inv = false, dep_visc = false;
    for (int p = 0; p < np; ++p) {
        int ci, cj;
        source_of(L, pi[p], pj[p], ci, cj);
        const bool hit = ci == si && cj == sj;
        if (p < 4) dep_inv = dep_inv || hit;
        if (p == 1 || p == 2 || p >= 4) dep_visc = dep_visc || hit;
    }
    const int NS = L.NS;
    const bool inL = interior(L, iL, jL), inR = interior(L, a, b);
    const int sL = L.slot(iL, jL);
    double mu[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double l = inL ? lam[k * NS + sL] / geo[G_VOL * NS + sL] : 0.0;
        const double r = inR ? lam[k * NS + sf] / geo[G_VOL * NS + sf] : 0.0;
        mu[k] = l - r;
    }
    Ctx c;
    make_ctx(c, L, geo, u, mut, ph);
    c.si = si;
    c.sj = sj;
    c.inv = dep_inv;
    c.viscous = ph.rans && dep_visc;
    const bool wall = !xi && b == 0 && !cut_col(L, a);
    D4 C[4], V[4];
    face<double>(c, iL, jL, a, b, iLL, jLL, iRR, jRR, xi, geo[(xi ? G_SXI_X : G_SETA_X) * NS + sf],
                 geo[(xi ? G_SXI_Y : G_SETA_Y) * NS + sf], wall, vAi, vAj, vBi, vBj, C, V);
    const int ts = L.slot(si, sj);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        double d[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) d[k] = part == 1 ? C[k].d[m] : part == 2 ? V[k].d[m] : C[k].d[m] + V[k].d[m];
        const double v = ((mu[0] * d[0] + mu[1] * d[1]) + mu[2] * d[2]) + mu[3] * d[3];
        atomicAdd(out + m * NS + ts, v);
    }
}

// Grid-node sensitivities (chain rule through the metrics).  The residual
// depends on the nodes only through the metric planes SXI, SETA, SB0-3, VOL,
// XC, YC (the eddy viscosity, and with it the wall distance, is frozen).
// gbar(p, slot) += sum_c lam_c . dF_c / dG(p, slot): every interior cell
// seeds the metric entries its residual reads, four per evaluation.
constexpr int N_GEO_ADJ = G_YC + 1;       // planes G_SXI_X .. G_YC
constexpr int MAX_GSEEDS = 96;

__global__ __launch_bounds__(TPB) void k_vjp_geo(Lay L, const double *geo, const double *u, const double *mut,
                                                 Phys ph, const double *lam, double *gbar) {
    const BlockXY cb = xcd_block();
    int s, i, j;
    if (!interior_cell(L, cb.x * blockDim.x + threadIdx.x, s, i, j)) return;
    const int NS = L.NS;
    double lc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) lc[k] = lam[k * NS + s];
    if (lc[0] == 0.0 && lc[1] == 0.0 && lc[2] == 0.0 && lc[3] == 0.0) return;
    Ctx c;
    make_ctx(c, L, geo, u, mut, ph);
    int ep[MAX_GSEEDS], es[MAX_GSEEDS], n = 0;
    auto add = [&](int p, int ii, int jj) {
        const int t = L.slot(ii, jj);
        for (int q = 0; q < n; ++q)
            if (ep[q] == p && es[q] == t) return;
        if (n < MAX_GSEEDS) {
            ep[n] = p;
            es[n] = t;
            ++n;
        }
    };
    // the cell's faces and volume
    add(G_SXI_X, i, j); add(G_SXI_Y, i, j); add(G_SXI_X, i + 1, j); add(G_SXI_Y, i + 1, j);
    add(G_SETA_X, i, j); add(G_SETA_Y, i, j); add(G_SETA_X, i, j + 1); add(G_SETA_Y, i, j + 1);
    add(G_VOL, i, j);
    // mean face vectors of the two cells of each face (spectral radii)
    const int nb[5][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, -1}, {0, 1}};
    for (int q = 0; q < 5; ++q)
        for (int p = G_SB0; p <= G_SB3; ++p) add(p, i + nb[q][0], j + nb[q][1]);
    // centres of the cells around the face vertices (viscous gradients)
    if (c.viscous)
        for (int dj = -1; dj <= 1; ++dj)
            for (int di = -1; di <= 1; ++di) {
                add(G_XC, i + di, j + dj);
                add(G_YC, i + di, j + dj);
            }
    // boundary normals of the ghost states in the stencil
    for (int dj = -2; dj <= 2; ++dj)
        for (int di = -2; di <= 2; ++di) {
            const int a = i + di, b = j + dj;
            if (interior(L, a, b)) continue;
            const int jc = min(max(b, 0), L.nj - 1);
            if (a < 0) { add(G_SXI_X, 0, jc); add(G_SXI_Y, 0, jc); }
            if (a >= L.ni) { add(G_SXI_X, L.ni, jc); add(G_SXI_Y, L.ni, jc); }
            const int ia = a < 0 ? -1 - a : (a >= L.ni ? L.ni - 1 - (a - L.ni) : a);
            if (b < 0 && !cut_col(L, ia) && !c.noslip) { add(G_SETA_X, ia, 0); add(G_SETA_Y, ia, 0); }
            if (b >= L.nj) { add(G_SETA_X, ia, L.nj); add(G_SETA_Y, ia, L.nj); }
        }
    for (int g = 0; g < n; g += 4) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            c.gp[k] = g + k < n ? ep[g + k] : -1;
            c.gs[k] = g + k < n ? es[g + k] : -1;
        }
        D4 F[4];
        cell_residual<D4>(c, i, j, F);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (g + k >= n) break;
            const double v = ((lc[0] * F[0].d[k] + lc[1] * F[1].d[k]) + lc[2] * F[2].d[k]) + lc[3] * F[3].d[k];
            atomicAdd(gbar + (size_t)ep[g + k] * NS + es[g + k], v);
        }
    }
}

// gbar += dC_L/dS of the wall faces (the force is -sum p_w S; p_w does not
// depend on the metrics for no-slip or slip walls): one thread per column
__global__ void k_forces_geo(Lay L, const double *geo, const double *u, Phys ph, double *gbar) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.ni || cut_col(L, i)) return;
    const int NS = L.NS;
    Ctx c;
    make_ctx(c, L, geo, u, nullptr, ph);
    D4 Ug[4], Ui[4];
    state<double>(c, i, -1, Ug);
    state<double>(c, i, 0, Ui);
    const double pw = (0.5 * (dpres(Ug) + dpres(Ui))).v;
    const double a = ph.alpha_deg * (M_PI / 180.0);
    const double q = 0.5 * (ph.mach * ph.mach * GAM);
    const int f = L.slot(i, 0);
    gbar[(size_t)G_SETA_X * NS + f] += pw * sin(a) / q;
    gbar[(size_t)G_SETA_Y * NS + f] += -pw * cos(a) / q;
}

// (dG/dX)^T gbar: every padded slot differentiates its metrics (faces
// stored there, the cell's volume, centre and mean face vectors, or the
// reflected centre and copied metrics of a ghost cell) with respect to the
// nodes they depend on, four coordinates per evaluation, and scatters into
// the node gradients dx, dy ((nj + 1) x (ni + 1), i fastest).
__global__ __launch_bounds__(TPB) void k_geo_nodes(Lay L, const double *xn, const double *yn,
                                                   const double *gbar, double *dx, double *dy) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    int i, j;
    if (!decode(L, s, i, j)) return;
    const int NS = L.NS, W = L.ni + 1;
    double gb[N_GEO_ADJ];
    bool any = false;
#pragma unroll
    for (int p = 0; p < N_GEO_ADJ; ++p) {
        gb[p] = gbar[(size_t)p * NS + s];
        any = any || gb[p] != 0.0;
    }
    if (!any) return;
    const bool iface = i >= 0 && i <= L.ni && j >= 0 && j < L.nj;
    const bool jface = i >= 0 && i < L.ni && j >= 0 && j <= L.nj;
    // dependency nodes
    int nd[16][2], nn = 0;
    {
        auto Xd = [&](int I, int J) { return xn[J * W + I]; };
        auto Yd = [&](int I, int J) { return yn[J * W + I]; };
        if (iface) { nd[nn][0] = i; nd[nn][1] = j; nd[nn + 1][0] = i; nd[nn + 1][1] = j + 1; nn += 2; }
        if (jface) { nd[nn][0] = i; nd[nn][1] = j; nd[nn + 1][0] = i + 1; nd[nn + 1][1] = j; nn += 2; }
        if (interior(L, i, j)) {
            nd[nn][0] = i; nd[nn][1] = j; nd[nn + 1][0] = i + 1; nd[nn + 1][1] = j;
            nd[nn + 2][0] = i; nd[nn + 2][1] = j + 1; nd[nn + 3][0] = i + 1; nd[nn + 3][1] = j + 1;
            nn += 4;
        } else {
            double cx, cy;
            int si, sj;
            g_centre<double>(L, Xd, Yd, i, j, cx, cy, si, sj, nd + nn, &nn);
        }
    }
    // unique (node, axis) coordinates
    int cI[32], cJ[32], cA[32], nc = 0;
    for (int q = 0; q < nn; ++q) {
        bool dup = false;
        for (int r = 0; r < q; ++r) dup = dup || (nd[r][0] == nd[q][0] && nd[r][1] == nd[q][1]);
        if (dup) continue;
        for (int ax = 0; ax < 2; ++ax) {
            cI[nc] = nd[q][0];
            cJ[nc] = nd[q][1];
            cA[nc] = ax;
            ++nc;
        }
    }
    for (int g = 0; g < nc; g += 4) {
        auto X = [&](int I, int J) {
            D4 v = dc(xn[J * W + I]);
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (g + k < nc && cA[g + k] == 0 && cI[g + k] == I && cJ[g + k] == J) v.d[k] = 1.0;
            return v;
        };
        auto Y = [&](int I, int J) {
            D4 v = dc(yn[J * W + I]);
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (g + k < nc && cA[g + k] == 1 && cI[g + k] == I && cJ[g + k] == J) v.d[k] = 1.0;
            return v;
        };
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        auto take = [&](double w, const D4 &v) {
            if (w == 0.0) return;
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[k] += w * v.d[k];
        };
        if (iface) {
            D4 sx, sy;
            g_iface<D4>(X, Y, i, j, sx, sy);
            take(gb[G_SXI_X], sx);
            take(gb[G_SXI_Y], sy);
        }
        if (jface) {
            D4 sx, sy;
            g_jface<D4>(X, Y, i, j, sx, sy);
            take(gb[G_SETA_X], sx);
            take(gb[G_SETA_Y], sy);
        }
        D4 vol, xc, yc, sb[4];
        if (interior(L, i, j)) {
            g_cell<D4>(X, Y, i, j, vol, xc, yc, sb);
        } else {
            int si, sj;
            g_centre<D4>(L, X, Y, i, j, xc, yc, si, sj);
            D4 xs, ys;
            g_cell<D4>(X, Y, si, sj, vol, xs, ys, sb);
        }
        take(gb[G_VOL], vol);
        take(gb[G_XC], xc);
        take(gb[G_YC], yc);
        take(gb[G_SB0], sb[0]);
        take(gb[G_SB1], sb[1]);
        take(gb[G_SB2], sb[2]);
        take(gb[G_SB3], sb[3]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (g + k >= nc) break;
            double *dst = cA[g + k] == 0 ? dx : dy;
            atomicAdd(dst + cJ[g + k] * W + cI[g + k], acc[k]);
        }
    }
}

// dF/dalpha (degrees) and dF/dM at fixed state: lane 0 alpha, lane 1 Mach
// (through the far-field state and mu_inf = M sqrt(gamma) / Re)
__global__ __launch_bounds__(TPB) void k_param_partials(Lay L, const double *geo, const double *u,
                                                        const double *mut, Phys ph, double reynolds,
                                                        double *dFa, double *dFm) {
    const BlockXY cb = xcd_block();
    int s, i, j;
    if (!interior_cell(L, cb.x * blockDim.x + threadIdx.x, s, i, j)) return;
    const int NS = L.NS;
    Ctx c;
    make_ctx(c, L, geo, u, mut, ph);
    const double V = ph.mach * sqrt(GAM);
    const double a = ph.alpha_deg * (M_PI / 180.0);
    const double da = M_PI / 180.0;
    D4 vx = dc(ph.uinf[1]), vy = dc(ph.uinf[2]);
    vx.d[0] = -V * sin(a) * da;
    vx.d[1] = sqrt(GAM) * cos(a);
    vy.d[0] = V * cos(a) * da;
    vy.d[1] = sqrt(GAM) * sin(a);
    c.uinf[1] = vx;
    c.uinf[2] = vy;
    D4 E = 0.5 * (vx * vx + vy * vy);
    c.uinf[3] = D4{ph.uinf[3], {E.d[0], E.d[1], 0.0, 0.0}};
    if (ph.rans) c.mu_inf.d[1] = sqrt(GAM) / reynolds;
    D4 F[4];
    cell_residual<double>(c, i, j, F);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        dFa[k * NS + s] = F[k].d[0];
        dFm[k * NS + s] = F[k].d[1];
    }
}

// Wall pressure force (the residual's own wall flux p_w S, p_w the mean of
// the wall cell and its ghost): one workgroup, deterministic tree sum.
// out[0..5] = C_L, C_D, dC_L/dalpha_deg, dC_L/dM (at fixed state), F_x, F_y;
// dcl (padded, zeroed) receives dC_L/du on the wall cells.
__global__ __launch_bounds__(TPB) void k_forces(Lay L, const double *geo, const double *u, Phys ph,
                                                double *out, double *dcl) {
    __shared__ double sx_[TPB], sy_[TPB];
    const int NS = L.NS;
    Ctx c;
    make_ctx(c, L, geo, u, nullptr, ph);
    const double a = ph.alpha_deg * (M_PI / 180.0);
    const double q = 0.5 * (ph.mach * ph.mach * GAM);
    double fx = 0.0, fy = 0.0;
    for (int i = threadIdx.x; i < L.ni; i += TPB) {
        if (cut_col(L, i)) continue;
        c.si = i;
        c.sj = 0;
        D4 Ug[4], Ui[4];
        state<double>(c, i, -1, Ug);
        state<double>(c, i, 0, Ui);
        D4 pw = 0.5 * (dpres(Ug) + dpres(Ui));
        const int f = L.slot(i, 0);
        const double Sx = geo[G_SETA_X * NS + f], Sy = geo[G_SETA_Y * NS + f];
        fx -= pw.v * Sx;
        fy -= pw.v * Sy;
        if (dcl) {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const double dfx = -pw.d[m] * Sx, dfy = -pw.d[m] * Sy;
                dcl[m * NS + f] = (dfy * cos(a) - dfx * sin(a)) / q;
            }
        }
    }
    sx_[threadIdx.x] = fx;
    sy_[threadIdx.x] = fy;
    __syncthreads();
    for (int w = TPB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sx_[threadIdx.x] += sx_[threadIdx.x + w];
            sy_[threadIdx.x] += sy_[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double Fx = sx_[0], Fy = sy_[0];
        const double cl = (Fy * cos(a) - Fx * sin(a)) / q;
        const double cd = (Fx * cos(a) + Fy * sin(a)) / q;
        out[0] = cl;
        out[1] = cd;
        out[2] = (-Fy * sin(a) - Fx * cos(a)) * (M_PI / 180.0) / q;
        out[3] = -2.0 * cl / ph.mach;
        out[4] = Fx;
        out[5] = Fy;
    }
}

// Transposed SGS preconditioner x = P^-T r, P = (D+L) D^-1 (D+U), with the
// stored D^-1 and M_s = D^-1 B_s: with zeta = D^T z and xi = D^T x,
//     ascending:  zeta_c = r_c  - sum_{nb earlier} M_{nb->c}^T zeta_nb
//     descending: xi_c   = zeta_c - sum_{nb later} M_{nb->c}^T xi_nb,
//                 x_c    = D_c^-T xi_c,
// where M_{nb->c} is neighbour nb's block toward c.  Both passes are the
// primal sweep's recurrences once cell c holds, in its own slot for the
// direction of nb, the block M_{nb->c}^T: k_blocks_t writes that array
// (the west slot of c holds the transposed east block of its west
// neighbour, and so on; on the wake cut of a C-grid, row-0 cells couple to
// their partner across the cut, whose south block is the one toward c), so
// the banded hyperplane sweep runs the solve with g = r and y = zeta, and
// k_dinv_t finishes with x = D^-T xi.
template <typename T>
__device__ inline void put_transposed(const T *blk, int bsrc, int ssrc, bool on, T *bt, int bdst, int NS, int s) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c)
            bt[BL<T>::at(bdst, NS, s, r, c)] = on ? blk[BL<T>::at(bsrc, NS, ssrc, c, r)] : (T)0;
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_blocks_t(Lay L, const T *blk, T *bt) {
    const BlockXY cb = xcd_block();
    int s, i, j;
    if (!interior_cell(L, cb.x * blockDim.x + threadIdx.x, s, i, j)) return;
    const int ni = L.ni, nj = L.nj, NS = L.NS, NJ = L.NJ, nw = L.nw;
    put_transposed(blk, B_M0 + 1, i > 0 ? s - NJ : s, i > 0, bt, B_M0 + 0, NS, s);            // west: its east block
    put_transposed(blk, B_M0 + 0, i < ni - 1 ? s + NJ : s, i < ni - 1, bt, B_M0 + 1, NS, s);  // east: its west block
    const bool cut = j == 0 && L.topo == 1 && (i < nw || i >= ni - nw);
    const int ss = j > 0 ? s - NJ - 1 : cut ? L.slot(ni - 1 - i, 0) : s;
    put_transposed(blk, j > 0 ? B_M0 + 3 : B_M0 + 2, ss, j > 0 || cut, bt, B_M0 + 2, NS, s);  // south (or partner)
    put_transposed(blk, B_M0 + 2, j < nj - 1 ? s + NJ + 1 : s, j < nj - 1, bt, B_M0 + 3, NS, s);  // north: its south block
}

// x = D^-T xi over the interior, in the blocks' precision
template <typename T>
__global__ __launch_bounds__(TPB) void k_dinv_t(Lay L, const T *blk, const double *xi, double *x) {
    const BlockXY cb = xcd_block();
    int s, i, j;
    if (!interior_cell(L, cb.x * blockDim.x + threadIdx.x, s, i, j)) return;
    const int NS = L.NS;
    T v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (T)xi[k * NS + s];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        T acc = (T)0;
#pragma unroll
        for (int k = 0; k < 4; ++k) acc = fma(blk[BL<T>::at(B_DINV, NS, s, k, rr)], v[k], acc);
        x[rr * NS + s] = (double)acc;
    }
}

// the sweep's input g = r in the sweep precision (interior cells)
template <typename T>
__global__ __launch_bounds__(TPB) void k_to_sweep(Lay L, const double *r, T *g) {
    const BlockXY cb = xcd_block();
    int s, i, j;
    if (!interior_cell(L, cb.x * blockDim.x + threadIdx.x, s, i, j)) return;
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k * L.NS + s] = (T)r[k * L.NS + s];
}

// sum of squares of all four components over the interior, and dot
// products; fixed-order two-pass reductions
constexpr int RB = 128;
__global__ __launch_bounds__(TPB) void k_dot1(Lay L, const double *a, const double *b, double *red) {
    __shared__ double sh[TPB];
    double acc = 0.0;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < L.NS; s += gridDim.x * blockDim.x) {
        int i, j;
        if (decode(L, s, i, j) && interior(L, i, j)) {
#pragma unroll
            for (int k = 0; k < 4; ++k) acc += a[k * L.NS + s] * b[k * L.NS + s];
        }
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = TPB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) red[blockIdx.x] = sh[0];
}

__global__ void k_dot2(const double *red, double *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0.0;
    for (int k = 0; k < RB; ++k) a += red[k];
    *out = a;
}

// out = a x + b y on the interior (four components), plain pointers
__global__ void k_axpby_p(Lay L, double a, const double *x, double b, const double *y, double *out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    int i, j;
    if (!decode(L, s, i, j) || !interior(L, i, j)) return;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int o = k * L.NS + s;
        out[o] = (y == nullptr) ? a * x[o] : a * x[o] + b * y[o];
    }
}

// out = x + a * dts * z (x may be null: out = a * dts * z)
// Transposes of the FAS transfers (Section 3) for the adjoint's coarse
// corrections.  The prolongation sets a fine correction to
// (9 e_parent + 3 e_i-neighbour + 3 e_j-neighbour + e_diagonal) / 16 of the
// coarse one (the parent standing in for a missing neighbour, the partner
// across the wake cut for a missing south one); its transpose adds each fine
// value with those weights to the same four coarse cells (atomically: the
// coarse cells are shared).
__global__ void k_adj_prolong_t(Lay Lf, Lay Lc, const double *lf, double *lc) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    int i, j;
    if (!decode(Lf, s, i, j) || !interior(Lf, i, j)) return;
    const int I = i / 2, J = j / 2;
    const int In = I + ((i & 1) ? 1 : -1), Jn = J + ((j & 1) ? 1 : -1);
    const bool vi = In >= 0 && In < Lc.ni, vj = Jn >= 0 && Jn < Lc.nj;
    const int s0 = Lc.slot(I, J);
    const int s1 = vi ? Lc.slot(In, J) : s0;
    int s2 = s0, s3 = s0;
    if (vj) s2 = Lc.slot(I, Jn);
    else if (Jn < 0 && cut_col(Lc, I)) s2 = Lc.slot(Lc.ni - 1 - I, 0);
    if (vi && vj) s3 = Lc.slot(In, Jn);
    else if (vi && Jn < 0 && cut_col(Lc, In)) s3 = Lc.slot(Lc.ni - 1 - In, 0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double v = lf[k * Lf.NS + s] * 0.0625;
        double *c = lc + (size_t)k * Lc.NS;
        atomicAdd(c + s0, 9.0 * v);
        atomicAdd(c + s1, 3.0 * v);
        atomicAdd(c + s2, 3.0 * v);
        atomicAdd(c + s3, v);
    }
}

// The restriction is the volume-weighted mean of the four children; its
// transpose adds V_fine / V_coarse times the parent's value to each child.
__global__ void k_adj_restrict_t(Lay Lf, Lay Lc, const double *geof, const double *geoc, const double *lc,
                                 double *lf) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    int i, j;
    if (!decode(Lf, s, i, j) || !interior(Lf, i, j)) return;
    const int sc = Lc.slot(i / 2, j / 2);
    const double w = geof[G_VOL * Lf.NS + s] / geoc[G_VOL * Lc.NS + sc];
#pragma unroll
    for (int k = 0; k < 4; ++k) lf[k * Lf.NS + s] += w * lc[k * Lc.NS + sc];
}

__global__ void k_adj_update(Lay L, const double *x, double a, const double *dts, const double *z,
                             double *out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    int i, j;
    if (!decode(L, s, i, j) || !interior(L, i, j)) return;
    const double d = dts[s];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int o = k * L.NS + s;
        out[o] = (x == nullptr) ? a * (d * z[o]) : x[o] + a * (d * z[o]);
    }
}

// out[i] = <w, v_i> for the n vectors v_i = basis + i * V (interior,
// four components); fixed-order two-pass reduction
__global__ __launch_bounds__(TPB) void k_mdot1(Lay L, const double *w, const double *basis, size_t V,
                                               double *red) {
    __shared__ double sh[TPB];
    const double *v = basis + (size_t)blockIdx.y * V;
    double acc = 0.0;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < L.NS; s += gridDim.x * blockDim.x) {
        int i, j;
        if (decode(L, s, i, j) && interior(L, i, j)) {
#pragma unroll
            for (int k = 0; k < 4; ++k) acc += w[k * L.NS + s] * v[k * L.NS + s];
        }
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int q = TPB / 2; q > 0; q >>= 1) {
        if ((int)threadIdx.x < q) sh[threadIdx.x] += sh[threadIdx.x + q];
        __syncthreads();
    }
    if (threadIdx.x == 0) red[(size_t)blockIdx.y * RB + blockIdx.x] = sh[0];
}

__global__ void k_mdot2(const double *red, int n, double *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a = 0.0;
    for (int k = 0; k < RB; ++k) a += red[(size_t)i * RB + k];
    out[i] = a;
}

// w -= sum_i h_i v_i
__global__ void k_maxpy(Lay L, double *w, const double *basis, size_t V, const double *h, int n) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    int i, j;
    if (!decode(L, s, i, j) || !interior(L, i, j)) return;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const size_t o = (size_t)k * L.NS + s;
        double a = w[o];
        for (int q = 0; q < n; ++q) a -= h[q] * basis[(size_t)q * V + o];
        w[o] = a;
    }
}

__global__ void k_zero(double *p, size_t n) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0.0;
}

}  // namespace

// =================================================================== launchers
void launch_vjp(const Lay &L, const double *geo, const double *u, const double *mut, const Phys &ph,
                const double *lam, double *out, hipStream_t st, int part) {
    const int nf = (L.ni + 1) * L.nj + L.ni * (L.nj + 1);
    hipLaunchKernelGGL(k_vjp, dim3(nblocks(nf), VJP_SOURCES), dim3(TPB), 0, st, L, geo, u, mut, ph, lam, out,
                       part);
}

void launch_param_partials(const Lay &L, const double *geo, const double *u, const double *mut,
                           const Phys &ph, double reynolds, double *dFa, double *dFm, hipStream_t st) {
    hipLaunchKernelGGL(k_param_partials, dim3(nblocks(L.ni * L.nj)), dim3(TPB), 0, st, L, geo, u, mut, ph,
                       reynolds, dFa, dFm);
}

void launch_vjp_geo(const Lay &L, const double *geo, const double *u, const double *mut, const Phys &ph,
                    const double *lam, double *gbar, hipStream_t st) {
    hipLaunchKernelGGL(k_vjp_geo, dim3(nblocks(L.ni * L.nj)), dim3(TPB), 0, st, L, geo, u, mut, ph, lam, gbar);
}

void launch_forces_geo(const Lay &L, const double *geo, const double *u, const Phys &ph, double *gbar,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_forces_geo, dim3(nblocks(L.ni)), dim3(TPB), 0, st, L, geo, u, ph, gbar);
}

void launch_geo_nodes(const Lay &L, const double *xn, const double *yn, const double *gbar, double *dx,
                      double *dy, hipStream_t st) {
    hipLaunchKernelGGL(k_geo_nodes, dim3(nblocks(L.NS)), dim3(TPB), 0, st, L, xn, yn, gbar, dx, dy);
}

void launch_forces(const Lay &L, const double *geo, const double *u, const Phys &ph, double *out,
                   double *dcl, hipStream_t st) {
    hipLaunchKernelGGL(k_forces, dim3(1), dim3(TPB), 0, st, L, geo, u, ph, out, dcl);
}

void launch_blocks_t(const Lay &L, const void *blk, void *bt, int fp32, hipStream_t st) {
    const dim3 g(nblocks(L.ni * L.nj)), b(TPB);
    if (fp32) hipLaunchKernelGGL(k_blocks_t<float>, g, b, 0, st, L, (const float *)blk, (float *)bt);
    else hipLaunchKernelGGL(k_blocks_t<double>, g, b, 0, st, L, (const double *)blk, (double *)bt);
}

void launch_to_sweep(const Lay &L, const double *r, void *g, int fp32, hipStream_t st) {
    const dim3 gr(nblocks(L.ni * L.nj)), b(TPB);
    if (fp32) hipLaunchKernelGGL(k_to_sweep<float>, gr, b, 0, st, L, r, (float *)g);
    else hipLaunchKernelGGL(k_to_sweep<double>, gr, b, 0, st, L, r, (double *)g);
}

void launch_dinv_t(const Lay &L, const void *blk, const double *xi, double *x, int fp32, hipStream_t st) {
    const dim3 g(nblocks(L.ni * L.nj)), b(TPB);
    if (fp32) hipLaunchKernelGGL(k_dinv_t<float>, g, b, 0, st, L, (const float *)blk, xi, x);
    else hipLaunchKernelGGL(k_dinv_t<double>, g, b, 0, st, L, (const double *)blk, xi, x);
}

int dot_scratch_size() { return RB; }

void launch_dot(const Lay &L, const double *a, const double *b, double *red, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_dot1, dim3(RB), dim3(TPB), 0, st, L, a, b, red);
    hipLaunchKernelGGL(k_dot2, dim3(1), dim3(64), 0, st, red, out);
}

void launch_axpby_ptr(const Lay &L, double a, const double *x, double b, const double *y, double *out,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_axpby_p, dim3(nblocks(L.NS)), dim3(TPB), 0, st, L, a, x, b, y, out);
}

void launch_adj_prolong_t(const Lay &Lf, const Lay &Lc, const double *lf, double *lc, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_prolong_t, dim3(nblocks(Lf.NS)), dim3(TPB), 0, st, Lf, Lc, lf, lc);
}

void launch_adj_restrict_t(const Lay &Lf, const Lay &Lc, const double *geof, const double *geoc, const double *lc,
                           double *lf, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_restrict_t, dim3(nblocks(Lf.NS)), dim3(TPB), 0, st, Lf, Lc, geof, geoc, lc, lf);
}

void launch_adj_update(const Lay &L, const double *x, double a, const double *dts, const double *z,
                       double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_update, dim3(nblocks(L.NS)), dim3(TPB), 0, st, L, x, a, dts, z, out);
}

void launch_mdot(const Lay &L, const double *w, const double *basis, size_t V, int n, double *red,
                 double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_mdot1, dim3(RB, n), dim3(TPB), 0, st, L, w, basis, V, red);
    hipLaunchKernelGGL(k_mdot2, dim3(nblocks(n, 64)), dim3(64), 0, st, red, n, out);
}

void launch_maxpy(const Lay &L, double *w, const double *basis, size_t V, const double *h, int n,
                  hipStream_t st) {
    hipLaunchKernelGGL(k_maxpy, dim3(nblocks(L.NS)), dim3(TPB), 0, st, L, w, basis, V, h, n);
}

void launch_zero(double *p, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + TPB - 1) / TPB)), dim3(TPB), 0, st, p, n);
}

}  // namespace fas
