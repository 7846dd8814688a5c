// Metrics of a level as functions of its node coordinates: Section 2
// (cell-centred finite volumes on a structured mesh; ghost cells mirror
// the interior cell across the boundary face, and across the C-grid wake
// cut the ghost is the partner cell).  Templated on the scalar, so the same
// expressions give the stored metrics (double) and their derivatives with
// respect to node coordinates (forward-mode dual numbers in the adjoint).
// X(I, J) and Y(I, J) return node coordinates; gsqrt must be overloaded
// for the scalar.
#pragma once
#include "fas_internal.h"

namespace fas {

__device__ inline double gsqrt(double v) { return sqrt(v); }

// i-face (I, j), from node (I, j) to (I, j + 1); points towards +i
template <class S, class XF, class YF>
__device__ inline void g_iface(XF X, YF Y, int I, int j, S &sx, S &sy) {
    S dx = X(I, j + 1) - X(I, j);
    S dy = Y(I, j + 1) - Y(I, j);
    sx = dy;
    sy = -dx;
}

// j-face (i, J), from node (i, J) to (i + 1, J); points towards +j
template <class S, class XF, class YF>
__device__ inline void g_jface(XF X, YF Y, int i, int J, S &sx, S &sy) {
    S dx = X(i + 1, J) - X(i, J);
    S dy = Y(i + 1, J) - Y(i, J);
    sx = -dy;
    sy = dx;
}

// interior cell (i, j): volume (half the cross product of the diagonals),
// centre (mean of the four nodes), mean i- and j-face vectors
template <class S, class XF, class YF>
__device__ inline void g_cell(XF X, YF Y, int i, int j, S &vol, S &xc, S &yc, S sb[4]) {
    S d1x = X(i + 1, j + 1) - X(i, j), d1y = Y(i + 1, j + 1) - Y(i, j);
    S d2x = X(i, j + 1) - X(i + 1, j), d2y = Y(i, j + 1) - Y(i + 1, j);
    vol = 0.5 * (d1x * d2y - d1y * d2x);
    xc = 0.25 * (((X(i, j) + X(i + 1, j)) + X(i + 1, j + 1)) + X(i, j + 1));
    yc = 0.25 * (((Y(i, j) + Y(i + 1, j)) + Y(i + 1, j + 1)) + Y(i, j + 1));
    S wx = Y(i, j + 1) - Y(i, j), wy = -(X(i, j + 1) - X(i, j));
    S ex = Y(i + 1, j + 1) - Y(i + 1, j), ey = -(X(i + 1, j + 1) - X(i + 1, j));
    S sx = -(Y(i + 1, j) - Y(i, j)), sy = X(i + 1, j) - X(i, j);
    S nx = -(Y(i + 1, j + 1) - Y(i, j + 1)), ny = X(i + 1, j + 1) - X(i, j + 1);
    sb[0] = 0.5 * (wx + ex);
    sb[1] = 0.5 * (wy + ey);
    sb[2] = 0.5 * (sx + nx);
    sb[3] = 0.5 * (sy + ny);
}

// (cx, cy) reflected across the line through (mx, my) normal to (sx, sy)
template <class S>
__device__ inline void g_reflect(S &cx, S &cy, S mx, S my, S sx, S sy) {
    S ln = gsqrt(sx * sx + sy * sy);
    S nx = sx / ln, ny = sy / ln;
    S dist = (cx - mx) * nx + (cy - my) * ny;
    cx = cx - 2.0 * dist * nx;
    cy = cy - 2.0 * dist * ny;
}

// Centre of padded cell (i, j), i in [0, ni), j in [-2, nj + 2), and the
// interior cell (si, sj) whose volume and mean face vectors it copies.
// Collects the nodes the centre depends on into nd (if given).
template <class S, class XF, class YF>
__device__ inline void g_jrow_centre(const Lay &L, XF X, YF Y, int i, int j, S &cx, S &cy, int &si, int &sj,
                                     int (*nd)[2] = nullptr, int *nn = nullptr) {
    S vol, sb[4];
    auto add = [&](int I, int J) {
        if (nd) {
            nd[*nn][0] = I;
            nd[*nn][1] = J;
            ++*nn;
        }
    };
    if (j >= 0 && j < L.nj) {
        si = i;
        sj = j;
        g_cell(X, Y, i, j, vol, cx, cy, sb);
        add(i, j); add(i + 1, j); add(i, j + 1); add(i + 1, j + 1);
        return;
    }
    if (j < 0) {
        const int k = -1 - j;
        if (L.topo == 1 && (i < L.nw || i >= L.ni - L.nw)) {     // wake cut: the partner cell
            si = L.ni - 1 - i;
            sj = k;
            g_cell(X, Y, si, sj, vol, cx, cy, sb);
            add(si, sj); add(si + 1, sj); add(si, sj + 1); add(si + 1, sj + 1);
            return;
        }
        si = i;
        sj = k;
        g_cell(X, Y, si, sj, vol, cx, cy, sb);
        S fx, fy;
        g_jface<S>(X, Y, i, 0, fx, fy);
        S mx = 0.5 * (X(i, 0) + X(i + 1, 0)), my = 0.5 * (Y(i, 0) + Y(i + 1, 0));
        g_reflect(cx, cy, mx, my, fx, fy);
        add(si, sj); add(si + 1, sj); add(si, sj + 1); add(si + 1, sj + 1);
        add(i, 0); add(i + 1, 0);
        return;
    }
    const int k = j - L.nj;
    si = i;
    sj = L.nj - 1 - k;
    g_cell(X, Y, si, sj, vol, cx, cy, sb);
    S fx, fy;
    g_jface<S>(X, Y, i, L.nj, fx, fy);
    S mx = 0.5 * (X(i, L.nj) + X(i + 1, L.nj)), my = 0.5 * (Y(i, L.nj) + Y(i + 1, L.nj));
    g_reflect(cx, cy, mx, my, fx, fy);
    add(si, sj); add(si + 1, sj); add(si, sj + 1); add(si + 1, sj + 1);
    add(i, L.nj); add(i + 1, L.nj);
}

// centre of any padded cell (i, j), i, j in [-2, n + 2): ghost columns
// reflect the mirrored column's centre across the i-boundary face
template <class S, class XF, class YF>
__device__ inline void g_centre(const Lay &L, XF X, YF Y, int i, int j, S &cx, S &cy, int &si, int &sj,
                                int (*nd)[2] = nullptr, int *nn = nullptr) {
    if (i >= 0 && i < L.ni) {
        g_jrow_centre(L, X, Y, i, j, cx, cy, si, sj, nd, nn);
        return;
    }
    const int jc = min(max(j, 0), L.nj - 1);
    const int isrc = i < 0 ? -1 - i : L.ni - 1 - (i - L.ni);
    const int I = i < 0 ? 0 : L.ni;
    g_jrow_centre(L, X, Y, isrc, j, cx, cy, si, sj, nd, nn);
    S fx, fy;
    g_iface<S>(X, Y, I, jc, fx, fy);
    S mx = 0.5 * (X(I, jc) + X(I, jc + 1)), my = 0.5 * (Y(I, jc) + Y(I, jc + 1));
    g_reflect(cx, cy, mx, my, fx, fy);
    if (nd) {
        nd[*nn][0] = I;
        nd[*nn][1] = jc;
        nd[*nn + 1][0] = I;
        nd[*nn + 1][1] = jc + 1;
        *nn += 2;
    }
}

}  // namespace fas
