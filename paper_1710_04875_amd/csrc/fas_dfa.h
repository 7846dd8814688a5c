// Discrete Fourier analysis of the preconditioned smoothers (Section
// "Discrete Fourier Analysis"): the per-case descriptor and the launcher.
#pragma once
#include <hip/hip_runtime.h>

namespace fas {

// discrete Fourier analysis: one case (linearisation state, scheme
// coefficients, mesh of phase angles, parameters); start = index of its
// first pair of phase angles in the concatenated output
struct DfaCase {
    double u[4];
    double alpha[5], beta[5];
    int s, wform, nx, ny, unsteady;
    int precond;      // 0: SGS, 1: exact D + L + U, 2: none
    int mesh;         // 0: dy = ar dx, 1: dy = dx / ar
    double cstar, d, eta, ar, c;
    long long start;
};
void launch_dfa(const DfaCase *d_cases, int n_cases, long long total, double *rad, double *amp, double *smooth,
                hipStream_t st);

}  // namespace fas
