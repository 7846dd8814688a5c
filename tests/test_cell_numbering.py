"""Host check of the hyperplane-ordered cell numbering that the cell-parallel
kernels launch over (rect_cell in fas_cells.h), and of the XCD-aware
renumbering of their workgroups (xcd_block).

The device functions and the layout struct are taken verbatim from the
sources, compiled for the host with g++, and run over every rectangle the
kernels use: interior cells, vertices and every padded cell, for all grids
up to 48 x 48 plus a few large and thin ones.  For each, the numbering must
hit every cell of the rectangle exactly once, give strictly increasing slots
(hyperplane order, j ascending inside a hyperplane), agree with decode(),
and reject numbers past the last cell; the workgroup renumbering must be a
bijection of every grid and hand one-row grids to the XCDs in runs, and the
column-group map of the eddy-viscosity launch (xcd_range) must be a
bijection that gives each XCD one contiguous range."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1710_04875_amd", "csrc")

MAIN = r"""
int main() {
    long bad = 0, checked = 0;
    auto run = [&](const Lay &L, int ri, int rj, int o) {
        std::vector<int> seen((size_t)ri * rj, 0);
        int last = -1;
        for (int t = 0; t < ri * rj + 70; ++t) {
            int s, i, j;
            const bool ok = rect_cell(L, t, ri, rj, o, s, i, j);
            if (t >= ri * rj) { if (ok) ++bad; continue; }
            int di, dj;
            if (!ok || i < -o || i >= ri - o || j < -o || j >= rj - o || s < 0 || s >= L.NS || s <= last ||
                !decode(L, s, di, dj) || di != i || dj != j) { ++bad; continue; }
            last = s;
            seen[(size_t)(i + o) * rj + (j + o)]++;
        }
        for (int v : seen) if (v != 1) ++bad;
        ++checked;
    };
    auto lay = [](int ni, int nj) {
        Lay L{};
        L.ni = ni; L.nj = nj; L.NI = ni + 2 * NG; L.NJ = nj + 2 * NG;
        L.NS = (L.NI + L.NJ - 1) * L.NJ;
        return L;
    };
    auto all = [&](int ni, int nj) {
        const Lay L = lay(ni, nj);
        run(L, ni, nj, 0);                 // interior cells
        run(L, ni + 1, nj + 1, 0);         // vertices
        run(L, L.NI, L.NJ, NG);            // every padded cell
        int s, i, j;                       // interior_cell is the interior rectangle
        for (int t = 0; t < ni * nj; t += 7) {
            int s2, i2, j2;
            if (!interior_cell(L, t, s, i, j) || !rect_cell(L, t, ni, nj, 0, s2, i2, j2) || s != s2) ++bad;
        }
    };
    for (int ni = 1; ni <= 48; ++ni)
        for (int nj = 1; nj <= 48; ++nj) all(ni, nj);
    const int big[][2] = {{512, 256}, {256, 512}, {1024, 64}, {16, 4096}, {4096, 8}};
    for (const auto &p : big) all(p[0], p[1]);
    // xcd_block: a bijection of every grid; one-row grids give each XCD
    // (hardware number w mod 8) whole runs of consecutive workgroups
    long grids = 0;
    const int gs[][2] = {{1, 1}, {7, 1}, {8, 1}, {9, 1}, {63, 1}, {64, 1}, {128, 1}, {511, 1}, {512, 1},
                         {513, 1}, {4096, 1}, {5000, 1}, {3, 5}, {512, 64}, {2048, 3}, {100, 7}};
    for (const auto &g : gs) {
        gridDim.x = g[0]; gridDim.y = g[1];
        const long G = (long)g[0] * g[1];
        std::vector<int> seen(G, 0), owner(G, -1);
        for (unsigned y = 0; y < gridDim.y; ++y)
            for (unsigned x = 0; x < gridDim.x; ++x) {
                blockIdx.x = x; blockIdx.y = y;
                const BlockXY b = xcd_block();
                if (b.x < 0 || b.x >= g[0] || b.y < 0 || b.y >= g[1]) { ++bad; continue; }
                const long v = (long)b.y * g[0] + b.x;
                seen[v]++;
                owner[v] = (int)((x + (long)y * g[0]) % XCD_COUNT);
            }
        for (int c : seen) if (c != 1) ++bad;
        if (g[1] == 1 && G >= (long)XCD_COUNT) {
            // inside the permuted rounds, runs of G / 8 (at most 64) share an XCD
            const long run = std::min<long>(XCD_RUN_MAX, G / XCD_COUNT);
            const long full = G / (XCD_COUNT * run) * (XCD_COUNT * run);
            for (long v = 0; v < full; ++v)
                if (owner[v] != owner[v - v % run]) ++bad;
        }
        ++grids;
    }
    // xcd_range: a bijection of every row width; for widths that are a
    // multiple of eight, XCD x mod 8 holds one contiguous range of gx / 8
    for (int gx = 1; gx <= 600; ++gx) {
        std::vector<int> seen(gx, 0), lo(XCD_COUNT, gx), hi(XCD_COUNT, -1);
        for (int x = 0; x < gx; ++x) {
            const int v = xcd_range(x, gx);
            if (v < 0 || v >= gx) { ++bad; continue; }
            seen[v]++;
            lo[x % XCD_COUNT] = std::min(lo[x % XCD_COUNT], v);
            hi[x % XCD_COUNT] = std::max(hi[x % XCD_COUNT], v);
        }
        for (int c : seen) if (c != 1) ++bad;
        if (gx % (int)XCD_COUNT == 0)
            for (unsigned x = 0; x < XCD_COUNT; ++x)
                if (hi[x] - lo[x] + 1 != gx / (int)XCD_COUNT || lo[x] != (int)x * (gx / (int)XCD_COUNT)) ++bad;
        ++grids;
    }
    std::printf("rectangles %ld grids %ld bad %ld\n", checked, grids, bad);
    return bad != 0;
}
"""


def _source():
    with open(os.path.join(CSRC, "fas_internal.h")) as f:
        internal = f.read()
    with open(os.path.join(CSRC, "fas_kernels.hip")) as f:
        kernels = f.read()
    ng = re.search(r"constexpr int NG = (\d+);", internal).group(1)
    lay = re.search(r"struct Lay \{.*?\n\};", internal, re.S).group(0)
    with open(os.path.join(CSRC, "fas_cells.h")) as f:
        cells = f.read()
    a = kernels.index("__device__ inline bool decode(")
    b = kernels.index("__device__ inline bool interior(const Lay &L, int i, int j) {")
    c = cells.index("__device__ inline int cells_before(")
    d = cells.rindex("}  // namespace fas")
    funcs = kernels[a:b] + cells[c:d]
    host = lambda t: t.replace("__host__ ", "").replace("__device__ ", "")
    head = ("#include <algorithm>\n#include <cmath>\n#include <cstdio>\n#include <vector>\n"
            "using std::max; using std::min;\nconstexpr int NG = %s;\n"
            "struct Dim3 { unsigned x = 0, y = 0; } gridDim, blockIdx;   // host stand-ins\n" % ng)
    return head + host(lay) + "\n" + host(funcs) + MAIN


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_rect_cell_numbering_is_a_hyperplane_ordered_bijection(tmp_path):
    src = tmp_path / "cells.cpp"
    exe = tmp_path / "cells"
    src.write_text(_source())
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("bad 0")
