// solve.hpp -- batched GMRES with iterative refinement over all frequencies and right-hand
// sides (solve.cpp) and its vector kernels (solve.hip).
#pragma once

#include <functional>

#include "common.hpp"

namespace bem {

// out[i][c] = <V_i[c], w[c]> for i < nvec (V_i at V + i vstride, columns of N entries)
void launch_dots(const zd* V, size_t vstride, int nvec, const zd* w, int N, int ncols, zd* out, hipStream_t st);
// w[c] += sign sum_{i < nvec} h[i][c] V_i[c]
void launch_combine(zd* w, const zd* V, size_t vstride, const zd* h, int nvec, int N, int ncols, double sign,
                    hipStream_t st);
// dst[c] = src[c] scale[c]
void launch_scale_cols(zd* dst, const zd* src, const double* scale, int N, int ncols, hipStream_t st);
// z = a x + b y over n entries
void launch_axpby(zd* z, double a, const zd* x, double b, const zd* y, size_t n, hipStream_t st);

// convolution quadrature in time: out[l] = W[l] + a v (W may be null), and the history
// recurrence W[l] = zinv[l] (W[l] + a v), over L rows of M entries
void launch_cq_fill(zd* out, const zd* W, const zd* v, double a, int L, int M, hipStream_t st);
void launch_cq_update(zd* W, const zd* v, const zd* zinv, double a, int L, int M, hipStream_t st);

// y = A x on device buffers [ncols][N]
using DevApply = std::function<void(const zd* x, zd* y)>;

struct SolveParams {
    double tol = 1e-8;        // ||b - A x|| <= tol ||b|| per column (fine operator)
    double inner_tol = 1e-3;  // relative residual of each inner GMRES run
    int restart = 30;
    int max_iter = 500;       // inner-operator applications in total
    int max_refine = 10;      // fine-operator residual evaluations after the first
};

struct SolveResult {
    int iterations = 0;
    int refinements = 0;
    double rel_residual = 0.0;
    bool converged = false;
};

// Solves A x = b column by column (ncols independent systems of size N) on device buffers:
// refinement sweeps r = b - A x (fine), inner GMRES(restart) on A_inner d = r, x += d.
SolveResult gmres_refine(const DevApply& A, const DevApply& A_inner, int N, int ncols, const zd* b, zd* x,
                         const SolveParams& p, hipStream_t st);

}  // namespace bem
