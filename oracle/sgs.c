/*
 * Block symmetric Gauss-Seidel application for the oracle (test
 * infrastructure only; never linked into the GPU library).
 *
 * Section 4.4, eq. "sgs-precon": P = (D + L) D^-1 (D + U) with 4x4 blocks.
 * P^-1 r is applied as
 *     forward,  ascending cell order:   y_c = D_c^-1 (r_c - sum_{nb<c} B_{c,nb} y_nb)
 *     backward, descending cell order:  x_c = D_c^-1 (D_c y_c - sum_{nb>c} B_{c,nb} x_nb)
 * The 4x4 diagonal solves use Gaussian elimination without pivoting, in a
 * fixed order (Section 4.4, last paragraph).
 *
 * Cells are numbered c = j*ni + i (lexicographic, i fastest).  Neighbour
 * slots: 0 west (i-1), 1 east (i+1), 2 south (j-1; for j = 0 in a C-grid
 * wake column, the partner cell across the cut), 3 north (j+1).
 * nb[c*4+s] holds the neighbour's cell number or -1 (boundary ghost:
 * coupling dropped).  Contributions are subtracted in slot order.
 * "Earlier" means a smaller cell number.
 *
 * Build: gcc -O2 -ffp-contract=off -shared -fPIC sgs.c -o libsgs_oracle.so
 */
#include <stddef.h>

static void solve4(const double *D, const double *rhs, double *x)
{
    double a[4][5];
    for (int r = 0; r < 4; ++r) {
        for (int c = 0; c < 4; ++c) a[r][c] = D[r * 4 + c];
        a[r][4] = rhs[r];
    }
    for (int k = 0; k < 4; ++k) {
        for (int r = k + 1; r < 4; ++r) {
            double f = a[r][k] / a[k][k];
            for (int c = k; c < 5; ++c) a[r][c] = a[r][c] - f * a[k][c];
        }
    }
    for (int r = 3; r >= 0; --r) {
        double s = a[r][4];
        for (int c = r + 1; c < 4; ++c) s = s - a[r][c] * x[c];
        x[r] = s / a[r][r];
    }
}

static void matvec_sub(const double *B, const double *v, double *acc)
{
    for (int r = 0; r < 4; ++r) {
        double s = 0.0;
        for (int c = 0; c < 4; ++c) s = s + B[r * 4 + c] * v[c];
        acc[r] = acc[r] - s;
    }
}

/* D: n*16, B: n*4*16, nb: n*4, r/y/x: n*4 (cell-major, 4 components) */
void sgs_forward(int n, const double *D, const double *B, const int *nb,
                 const double *r, double *y)
{
    for (int c = 0; c < n; ++c) {
        double acc[4];
        for (int k = 0; k < 4; ++k) acc[k] = r[c * 4 + k];
        for (int s = 0; s < 4; ++s) {
            int m = nb[c * 4 + s];
            if (m >= 0 && m < c) matvec_sub(B + ((size_t)c * 4 + s) * 16, y + (size_t)m * 4, acc);
        }
        solve4(D + (size_t)c * 16, acc, y + (size_t)c * 4);
    }
}

void sgs_backward(int n, const double *D, const double *B, const int *nb,
                  const double *y, double *x)
{
    for (int c = n - 1; c >= 0; --c) {
        double acc[4];
        const double *Dc = D + (size_t)c * 16;
        for (int r = 0; r < 4; ++r) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s = s + Dc[r * 4 + k] * y[c * 4 + k];
            acc[r] = s;
        }
        for (int s = 0; s < 4; ++s) {
            int m = nb[c * 4 + s];
            if (m > c) matvec_sub(B + ((size_t)c * 4 + s) * 16, x + (size_t)m * 4, acc);
        }
        solve4(Dc, acc, x + (size_t)c * 4);
    }
}

/* Same forward solve, visiting cells hyperplane by hyperplane (h = i + j
 * ascending, j ascending inside a hyperplane).  Used to show that the
 * result does not depend on which dependency-respecting order is taken. */
void sgs_forward_hyperplane(int ni, int nj, const double *D, const double *B,
                            const int *nb, const double *r, double *y)
{
    for (int h = 0; h < ni + nj - 1; ++h) {
        for (int j = 0; j < nj; ++j) {
            int i = h - j;
            if (i < 0 || i >= ni) continue;
            int c = j * ni + i;
            double acc[4];
            for (int k = 0; k < 4; ++k) acc[k] = r[c * 4 + k];
            for (int s = 0; s < 4; ++s) {
                int m = nb[c * 4 + s];
                if (m >= 0 && m < c) matvec_sub(B + ((size_t)c * 4 + s) * 16, y + (size_t)m * 4, acc);
            }
            solve4(D + (size_t)c * 16, acc, y + (size_t)c * 4);
        }
    }
}
