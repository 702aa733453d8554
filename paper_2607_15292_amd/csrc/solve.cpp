// solve.cpp -- batched GMRES with FP64 re-orthogonalised classical Gram-Schmidt and iterative
// refinement, for the systems V(s_l) t_l = (I/2 + K(s_l)) g_l of all frequencies and
// right-hand sides at once.  The Krylov vectors, products and inner products stay on the
// device; the small Hessenberg least-squares problems (Givens rotations) of every column are
// solved on the host after each Arnoldi step.
#include "solve.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

#include "host.hpp"

namespace bem {

namespace {

inline std::complex<double> tc(zd v) { return {v.re, v.im}; }
inline zd fc(std::complex<double> v) { return {v.real(), v.imag()}; }

// column norms ||w[c]|| into host memory
void col_norms(const zd* w, int N, int ncols, DevBuf& tmp, std::vector<double>& out, hipStream_t st)
{
    launch_dots(w, 0, 1, w, N, ncols, tmp.as<zd>(), st);
    std::vector<zd> h(ncols);
    BEM_HIP_TRY(hipMemcpyAsync(h.data(), tmp.p, ncols * sizeof(zd), hipMemcpyDeviceToHost, st));
    BEM_HIP_TRY(hipStreamSynchronize(st));
    out.resize(ncols);
    for (int c = 0; c < ncols; ++c) out[c] = std::sqrt(std::max(h[c].re, 0.0));
}

// One restarted-GMRES run on A d = r to ||r - A d|| <= rtol ||r|| per column (d starts at 0).
// Returns the operator applications used.
int gmres(const DevApply& A, int N, int ncols, const zd* r, zd* d, double rtol, int restart, int budget,
          hipStream_t st)
{
    const size_t vs = (size_t)N * ncols;
    const int m = std::max(1, restart);
    DevBuf basis, wbuf, res, hbuf, sbuf, nbuf;
    basis.alloc((size_t)(m + 1) * vs * sizeof(zd));
    wbuf.alloc(vs * sizeof(zd));
    res.alloc(vs * sizeof(zd));
    hbuf.alloc((size_t)(m + 1) * ncols * sizeof(zd));
    sbuf.alloc((size_t)ncols * sizeof(double));
    nbuf.alloc((size_t)ncols * sizeof(zd));
    zd* V = basis.as<zd>();
    zd* w = wbuf.as<zd>();
    zd* rr = res.as<zd>();
    BEM_HIP_TRY(hipMemsetAsync(d, 0, vs * sizeof(zd), st));
    std::vector<double> rnorm0, beta;
    col_norms(r, N, ncols, hbuf, rnorm0, st);
    int used = 0;
    bool first = true;
    while (used < budget) {
        // residual of the current d
        if (first) {
            BEM_HIP_TRY(hipMemcpyAsync(rr, r, vs * sizeof(zd), hipMemcpyDeviceToDevice, st));
        } else {
            A(d, w);
            ++used;
            launch_axpby(rr, 1.0, r, -1.0, w, vs, st);
        }
        first = false;
        col_norms(rr, N, ncols, hbuf, beta, st);
        bool done = true;
        std::vector<double> sc(ncols);
        std::vector<int> active(ncols);
        for (int c = 0; c < ncols; ++c) {
            active[c] = beta[c] > rtol * rnorm0[c] && beta[c] > 0.0;
            if (active[c]) done = false;
            sc[c] = active[c] ? 1.0 / beta[c] : 0.0;
        }
        if (done || used >= budget) break;
        BEM_HIP_TRY(hipMemcpyAsync(sbuf.p, sc.data(), ncols * sizeof(double), hipMemcpyHostToDevice, st));
        launch_scale_cols(V, rr, sbuf.as<double>(), N, ncols, st);
        // Hessenberg columns, rotations and the rotated right-hand side g per column
        std::vector<std::complex<double>> H((size_t)ncols * (m + 1) * m, 0.0), g((size_t)ncols * (m + 1), 0.0);
        std::vector<std::complex<double>> cs((size_t)ncols * m), sn((size_t)ncols * m);
        std::vector<int> kdone(ncols, 0);
        std::vector<char> fin(ncols, 0);  // column converged (or broke down) in this cycle
        for (int c = 0; c < ncols; ++c) g[(size_t)c * (m + 1)] = active[c] ? beta[c] : 0.0;
        std::vector<zd> h1((size_t)(m + 1) * ncols), h2((size_t)(m + 1) * ncols);
        int k = 0;
        for (; k < m && used < budget; ++k) {
            zd* Vk = V + (size_t)k * vs;
            A(Vk, w);
            ++used;
            // classical Gram-Schmidt, twice
            launch_dots(V, vs, k + 1, w, N, ncols, hbuf.as<zd>(), st);
            BEM_HIP_TRY(hipMemcpyAsync(h1.data(), hbuf.p, (size_t)(k + 1) * ncols * sizeof(zd), hipMemcpyDeviceToHost, st));
            launch_combine(w, V, vs, hbuf.as<zd>(), k + 1, N, ncols, -1.0, st);
            launch_dots(V, vs, k + 1, w, N, ncols, hbuf.as<zd>(), st);
            BEM_HIP_TRY(hipMemcpyAsync(h2.data(), hbuf.p, (size_t)(k + 1) * ncols * sizeof(zd), hipMemcpyDeviceToHost, st));
            launch_combine(w, V, vs, hbuf.as<zd>(), k + 1, N, ncols, -1.0, st);
            std::vector<double> hn;
            col_norms(w, N, ncols, nbuf, hn, st);  // synchronises: h1, h2 are on the host
            bool all = true;
            for (int c = 0; c < ncols; ++c) {
                if (!active[c] || fin[c]) {
                    sc[c] = 0.0;
                    continue;
                }
                std::complex<double>* Hc = &H[((size_t)c * m + k) * (m + 1)];  // column k of column c
                for (int i = 0; i <= k; ++i) Hc[i] = tc(h1[(size_t)i * ncols + c]) + tc(h2[(size_t)i * ncols + c]);
                Hc[k + 1] = hn[c];
                // previous rotations, then a new one zeroing Hc[k + 1]
                for (int i = 0; i < k; ++i) {
                    const std::complex<double> a = Hc[i], b = Hc[i + 1];
                    const std::complex<double> ci = cs[(size_t)c * m + i], si = sn[(size_t)c * m + i];
                    Hc[i] = std::conj(ci) * a + std::conj(si) * b;
                    Hc[i + 1] = -si * a + ci * b;
                }
                const double na = std::abs(Hc[k]), nb = std::abs(Hc[k + 1]);
                const double nr = std::hypot(na, nb);
                std::complex<double> ck = 1.0, sk = 0.0;
                if (nr > 0.0) {
                    ck = Hc[k] / nr;
                    sk = Hc[k + 1] / nr;
                }
                cs[(size_t)c * m + k] = ck;
                sn[(size_t)c * m + k] = sk;
                Hc[k] = nr;
                Hc[k + 1] = 0.0;
                std::complex<double>* gc = &g[(size_t)c * (m + 1)];
                const std::complex<double> gk = gc[k];
                gc[k] = std::conj(ck) * gk;
                gc[k + 1] = -sk * gk;
                kdone[c] = k + 1;
                const bool conv = std::abs(gc[k + 1]) <= rtol * rnorm0[c] || hn[c] <= 1e-14 * beta[c];
                sc[c] = conv || hn[c] <= 0.0 ? 0.0 : 1.0 / hn[c];
                fin[c] = conv;
                if (!conv) all = false;
            }
            BEM_HIP_TRY(hipMemcpyAsync(sbuf.p, sc.data(), ncols * sizeof(double), hipMemcpyHostToDevice, st));
            launch_scale_cols(V + (size_t)(k + 1) * vs, w, sbuf.as<double>(), N, ncols, st);
            if (all) {
                ++k;
                break;
            }
        }
        // y_c = R_c^{-1} g_c over the kdone[c] steps of column c; d += V y
        std::vector<zd> y((size_t)(m + 1) * ncols, zd{0.0, 0.0});
        for (int c = 0; c < ncols; ++c) {
            const int kc = kdone[c];
            std::vector<std::complex<double>> yc(kc);
            for (int i = kc - 1; i >= 0; --i) {
                std::complex<double> s = g[(size_t)c * (m + 1) + i];
                for (int j = i + 1; j < kc; ++j) s -= H[((size_t)c * m + j) * (m + 1) + i] * yc[j];
                const std::complex<double> dg = H[((size_t)c * m + i) * (m + 1) + i];
                yc[i] = std::abs(dg) > 0.0 ? s / dg : 0.0;
            }
            for (int i = 0; i < kc; ++i) y[(size_t)i * ncols + c] = fc(yc[i]);
        }
        BEM_HIP_TRY(hipMemcpyAsync(hbuf.p, y.data(), (size_t)(m + 1) * ncols * sizeof(zd), hipMemcpyHostToDevice, st));
        launch_combine(d, V, vs, hbuf.as<zd>(), std::max(k, 1), N, ncols, 1.0, st);
        BEM_HIP_TRY(hipStreamSynchronize(st));
    }
    return used;
}

}  // namespace

SolveResult gmres_refine(const DevApply& A, const DevApply& A_inner, int N, int ncols, const zd* b, zd* x,
                         const SolveParams& p, hipStream_t st)
{
    SolveResult R;
    const size_t vs = (size_t)N * ncols;
    DevBuf rbuf, dbuf, ybuf, tmp;
    rbuf.alloc(vs * sizeof(zd));
    dbuf.alloc(vs * sizeof(zd));
    ybuf.alloc(vs * sizeof(zd));
    tmp.alloc((size_t)std::max(ncols, 1) * sizeof(zd));
    zd* r = rbuf.as<zd>();
    zd* d = dbuf.as<zd>();
    zd* y = ybuf.as<zd>();
    std::vector<double> bn, rn;
    col_norms(b, N, ncols, tmp, bn, st);
    BEM_HIP_TRY(hipMemsetAsync(x, 0, vs * sizeof(zd), st));
    BEM_HIP_TRY(hipMemcpyAsync(r, b, vs * sizeof(zd), hipMemcpyDeviceToDevice, st));
    for (int sweep = 0;; ++sweep) {
        col_norms(r, N, ncols, tmp, rn, st);
        double worst = 0.0;
        for (int c = 0; c < ncols; ++c) worst = std::max(worst, bn[c] > 0.0 ? rn[c] / bn[c] : 0.0);
        R.rel_residual = worst;
        if (worst <= p.tol) {
            R.converged = true;
            break;
        }
        if (sweep > p.max_refine || R.iterations >= p.max_iter) break;
        // inner run: tight enough to reach tol in this sweep when the inner operator is the
        // fine one, else inner_tol
        double rtol = p.inner_tol;
        if (&A_inner == &A || p.inner_tol <= 0.0) rtol = std::max(0.5 * p.tol / std::max(worst, 1e-300), 1e-15);
        R.iterations += gmres(A_inner, N, ncols, r, d, std::min(rtol, 0.5), p.restart, p.max_iter - R.iterations, st);
        launch_axpby(x, 1.0, x, 1.0, d, vs, st);
        A(x, y);
        ++R.refinements;
        launch_axpby(r, 1.0, b, -1.0, y, vs, st);
    }
    BEM_HIP_TRY(hipStreamSynchronize(st));
    return R;
}

}  // namespace bem
