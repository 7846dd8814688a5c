// Numbering of the cells of a rectangle of a level in hyperplane order, for
// kernels that launch one thread per cell rather than one per padded slot.
#pragma once
#include "fas_internal.h"

namespace fas {

// Cell number t of the ri x rj rectangle of cells (i, j), -o <= i < ri - o,
// -o <= j < rj - o, in hyperplane order (h = i + j ascending, j ascending
// inside a hyperplane): consecutive t are consecutive slots of a hyperplane,
// so a wave's accesses stay coalesced while every lane holds a cell.  With
// m = min(ri, rj) and M = max(ri, rj), hyperplanes 0 .. m-2 of the rectangle
// hold 1 .. m-1 cells, m-1 .. M-1 hold m each and M .. ri+rj-2 hold m-1 .. 1;
// the hyperplane of t comes from inverting those prefix sums (a square root
// for the two triangles, then an exact integer check).
__device__ inline int cells_before(int h, int ri, int rj) {
    const int m = min(ri, rj), M = max(ri, rj);
    if (h <= m - 1) return h * (h + 1) / 2;
    const int A = (m - 1) * m / 2;
    if (h <= M) return A + (h - (m - 1)) * m;
    const int k = h - M;
    return A + (M - m + 1) * m + k * (m - 1) - k * (k - 1) / 2;
}
__device__ inline int tri_root(int t) {
    // largest h with h (h + 1) / 2 <= t
    int h = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((h + 1) * (h + 2) / 2 <= t) ++h;
    while (h * (h + 1) / 2 > t) --h;
    return h;
}
__device__ inline bool rect_cell(const Lay &L, int t, int ri, int rj, int o, int &s, int &i, int &j) {
    const int n = ri * rj;
    if (t >= n) return false;
    const int m = min(ri, rj), M = max(ri, rj);
    const int A = (m - 1) * m / 2, B = A + (M - m + 1) * m;
    int h;
    if (t < A) h = tri_root(t);
    else if (t < B) h = (m - 1) + (t - A) / m;
    else h = (ri + rj - 2) - tri_root(n - 1 - t);   // the last triangle, counted from the end
    const int jr = max(0, h - ri + 1) + (t - cells_before(h, ri, rj));
    i = h - jr - o;
    j = jr - o;
    s = L.slot(i, j);
    return true;
}
// Workgroups of a launch go to the eight XCDs in turn by linear number, and
// each XCD has its own L2.  For a launch over one grid (gridDim.y == 1)
// xcd_block renumbers the workgroups so that each XCD takes runs of
// consecutive ones instead: cells of neighbouring hyperplanes, whose
// stencils share states and metrics, then meet in one L2 rather than being
// fetched once per XCD.  Complete rounds of eight runs are permuted and the
// remaining workgroups keep their numbers; the map is a bijection, so it
// changes which workgroup computes a cell and nothing else.  Batched
// launches (one grid row per case, padded to the largest case) keep the
// hardware's order: there the real work sits at the start of every row, and
// runs would hand it to a few XCDs (measured: fewer HBM bytes, longer
// launches).
constexpr unsigned XCD_COUNT = 8, XCD_RUN_MAX = 64;
struct BlockXY {
    int x, y;
};
__device__ inline BlockXY xcd_block() {
    const unsigned gx = gridDim.x, G = gx * gridDim.y;
    const unsigned w = blockIdx.x + blockIdx.y * gx;
    const unsigned run = gridDim.y == 1 ? min(XCD_RUN_MAX, G / XCD_COUNT) : 0;
    unsigned v = w;
    if (run > 0 && w < G / (XCD_COUNT * run) * (XCD_COUNT * run)) {
        const unsigned x = w % XCD_COUNT, k = w / XCD_COUNT;
        v = ((k / run) * XCD_COUNT + x) * run + k % run;
    }
    return {(int)(v % gx), (int)(v / gx)};
}

// Column groups of the Baldwin-Lomax launch: a row of gx workgroups per
// grid, gx a multiple of eight, so workgroup x of the row runs on XCD
// x mod 8.  That XCD takes the contiguous range [(x mod 8) gx/8,
// (x mod 8 + 1) gx/8) of column groups, whose cells share cache lines at
// the range's interior; other widths keep their numbers.  A bijection of
// 0 .. gx - 1.
__device__ inline int xcd_range(int x, int gx) {
    return gx % (int)XCD_COUNT == 0 ? x % (int)XCD_COUNT * (gx / (int)XCD_COUNT) + x / (int)XCD_COUNT : x;
}

// interior cells: 0 <= i < ni, 0 <= j < nj
__device__ inline bool interior_cell(const Lay &L, int t, int &s, int &i, int &j) {
    return rect_cell(L, t, L.ni, L.nj, 0, s, i, j);
}

}  // namespace fas
