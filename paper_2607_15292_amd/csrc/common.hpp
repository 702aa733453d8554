// common.hpp -- complex arithmetic, 3x3 complex block helpers and HIP error plumbing
// shared by the libbem translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define BEM_HD __host__ __device__ __forceinline__

template <typename T>
struct cx {
    T re, im;
};

template <typename T> BEM_HD cx<T> mkc(T r, T i) { return cx<T>{r, i}; }
template <typename T> BEM_HD cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> BEM_HD cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> BEM_HD cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
template <typename T> BEM_HD cx<T> operator*(cx<T> a, cx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> BEM_HD cx<T> operator*(T a, cx<T> b) { return {a * b.re, a * b.im}; }
template <typename T> BEM_HD cx<T> operator*(cx<T> b, T a) { return {a * b.re, a * b.im}; }
template <typename T> BEM_HD cx<T>& operator+=(cx<T>& a, cx<T> b)
{
    a.re += b.re;
    a.im += b.im;
    return a;
}
template <typename T> BEM_HD cx<T>& operator-=(cx<T>& a, cx<T> b)
{
    a.re -= b.re;
    a.im -= b.im;
    return a;
}
template <typename T> BEM_HD cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
template <typename T> BEM_HD T abs2(cx<T> a) { return a.re * a.re + a.im * a.im; }
// a * conj(b)
template <typename T> BEM_HD cx<T> mul_conj(cx<T> a, cx<T> b)
{
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// conj(a) * b
template <typename T> BEM_HD cx<T> conj_mul(cx<T> a, cx<T> b)
{
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
BEM_HD float fma_r(float a, float b, float c) { return fmaf(a, b, c); }
BEM_HD double fma_r(double a, double b, double c) { return fma(a, b, c); }
// a * b + c as two fused multiply-adds per part (the accumulator enters the inner one)
template <typename T> BEM_HD cx<T> fma_c(cx<T> a, cx<T> b, cx<T> c)
{
    return {fma_r(a.re, b.re, fma_r(-a.im, b.im, c.re)), fma_r(a.re, b.im, fma_r(a.im, b.re, c.im))};
}

template <typename To, typename Ti> BEM_HD cx<To> cvt(cx<Ti> a) { return {(To)a.re, (To)a.im}; }

typedef cx<double> zd;
typedef cx<float> zf;

// ---------------------------------------------------------------- 3x3 complex blocks
// Row-major 3x3 blocks of complex<double>.

struct blk {
    zd a[9];
};

BEM_HD blk blk_zero()
{
    blk b;
#pragma unroll
    for (int t = 0; t < 9; ++t) b.a[t] = {0.0, 0.0};
    return b;
}

// C = A * B
BEM_HD blk blk_mul(const blk& A, const blk& B)
{
    blk C;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            zd s = A.a[3 * i] * B.a[j];
            s = fma_c(A.a[3 * i + 1], B.a[3 + j], s);
            s = fma_c(A.a[3 * i + 2], B.a[6 + j], s);
            C.a[3 * i + j] = s;
        }
    return C;
}

// C += A * B
BEM_HD void blk_mul_add(blk& C, const blk& A, const blk& B)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            zd s = C.a[3 * i + j];
            s = fma_c(A.a[3 * i], B.a[j], s);
            s = fma_c(A.a[3 * i + 1], B.a[3 + j], s);
            s = fma_c(A.a[3 * i + 2], B.a[6 + j], s);
            C.a[3 * i + j] = s;
        }
}

// C -= A * B
BEM_HD void blk_mul_sub(blk& C, const blk& A, const blk& B)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            zd s = A.a[3 * i] * B.a[j];
            s = fma_c(A.a[3 * i + 1], B.a[3 + j], s);
            s = fma_c(A.a[3 * i + 2], B.a[6 + j], s);
            C.a[3 * i + j] -= s;
        }
}

BEM_HD double blk_fro2(const blk& A)
{
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < 9; ++t) s += abs2(A.a[t]);
    return s;
}

// determinant and adjugate (transpose of the cofactor matrix): A * adj(A) = det(A) I
BEM_HD zd blk_det_adj(const blk& A, blk& adj)
{
    const zd* m = A.a;
    adj.a[0] = m[4] * m[8] - m[5] * m[7];
    adj.a[1] = m[2] * m[7] - m[1] * m[8];
    adj.a[2] = m[1] * m[5] - m[2] * m[4];
    adj.a[3] = m[5] * m[6] - m[3] * m[8];
    adj.a[4] = m[0] * m[8] - m[2] * m[6];
    adj.a[5] = m[2] * m[3] - m[0] * m[5];
    adj.a[6] = m[3] * m[7] - m[4] * m[6];
    adj.a[7] = m[1] * m[6] - m[0] * m[7];
    adj.a[8] = m[0] * m[4] - m[1] * m[3];
    return m[0] * adj.a[0] + m[1] * adj.a[3] + m[2] * adj.a[6];
}

BEM_HD zd zdiv(zd a, zd b)
{
    double d = 1.0 / (b.re * b.re + b.im * b.im);
    return {(a.re * b.re + a.im * b.im) * d, (a.im * b.re - a.re * b.im) * d};
}

// A power of two within a factor 2 of the largest |entry| of A (1 for a zero or non-finite
// block).  Scaling by it is exact, so a result computed on A / s and rescaled is the one
// computed on A wherever the latter does not underflow: entries of faces at the largest |s_l|
// reach exp(-Re(s) r / c2) ~ 1e-60, where det(A) ~ 1e-180 and its square underflow.
BEM_HD double blk_pow2_scale(const blk& A)
{
    double m = 0.0;
#pragma unroll
    for (int t = 0; t < 9; ++t) m = fmax(m, fmax(fabs(A.a[t].re), fabs(A.a[t].im)));
    if (!(m > 0.0) || !(m < 1e300)) return 1.0;
    int e;
    (void)frexp(m, &e);
    return ldexp(1.0, e);
}

BEM_HD blk blk_inv(const blk& A)
{
    const double sc = blk_pow2_scale(A), isc = 1.0 / sc;
    blk As;
#pragma unroll
    for (int t = 0; t < 9; ++t) As.a[t] = A.a[t] * isc;
    blk adj;
    zd det = blk_det_adj(As, adj);
    zd inv = zdiv(zd{isc, 0.0}, det);
#pragma unroll
    for (int t = 0; t < 9; ++t) adj.a[t] = adj.a[t] * inv;
    return adj;
}

// Largest eigenvalue of a 3x3 Hermitian positive semidefinite matrix M (row-major),
// trigonometric solution of the characteristic cubic (accurate in relative terms for the
// largest eigenvalue).
BEM_HD double herm3_lambda_max(const blk& M)
{
    double a = M.a[0].re, b = M.a[4].re, c = M.a[8].re;
    double p1 = abs2(M.a[1]) + abs2(M.a[2]) + abs2(M.a[5]);
    double q = (a + b + c) / 3.0;
    double aq = a - q, bq = b - q, cq = c - q;
    double p2 = aq * aq + bq * bq + cq * cq + 2.0 * p1;
    if (!(p2 > 1e-300 * (q * q + 1e-300))) return q;  // multiple of the identity
    double p = sqrt(p2 / 6.0);
    double ip = 1.0 / p;
    // B = (M - q I) / p; det(B) / 2
    zd b00 = {aq * ip, 0.0}, b11 = {bq * ip, 0.0}, b22 = {cq * ip, 0.0};
    zd b01 = M.a[1] * ip, b02 = M.a[2] * ip, b12 = M.a[5] * ip;
    zd b10 = conj(b01), b20 = conj(b02), b21 = conj(b12);
    zd det = b00 * (b11 * b22 - b12 * b21) - b01 * (b10 * b22 - b12 * b20) + b02 * (b10 * b21 - b11 * b20);
    double r = 0.5 * det.re;
    r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
    double phi = acos(r) / 3.0;
    return q + 2.0 * p * cos(phi);
}

// |r_33| of the Householder QR of a 3x3 complex block with column pivoting: after the first
// reflection (the column of largest norm) the trailing 2 x 2 block B has |r_22 r_33| =
// |det B| and |r_22| = the larger column norm of B.  Backward stable (errs by about
// eps ||A||) and never below sigma_3 (sigma_3 <= ||R_22||, here |r_33|).
template <int P>
BEM_HD double blk_r33_piv(const blk& A, double al)
{
    // pivot column x = A e_P, the other two columns y = A e_Q, z = A e_R (static indices: no
    // copies of the block, no indexed access)
    constexpr int Q = P == 0 ? 1 : 0, R = P == 2 ? 1 : 2;
    // v = x + e^{i arg x_0} ||x|| e_0, H = I - 2 v v^H / (v^H v)
    const zd x0 = A.a[P];
    const double a0 = sqrt(abs2(x0));
    const zd v0 = x0 + (a0 > 0.0 ? x0 * (al / a0) : zd{al, 0.0});
    const zd v1 = A.a[3 + P], v2 = A.a[6 + P];
    const double g = 2.0 / (abs2(v0) + abs2(v1) + abs2(v2));
    const zd fy = (conj_mul(v0, A.a[Q]) + conj_mul(v1, A.a[3 + Q]) + conj_mul(v2, A.a[6 + Q])) * g;
    const zd fz = (conj_mul(v0, A.a[R]) + conj_mul(v1, A.a[3 + R]) + conj_mul(v2, A.a[6 + R])) * g;
    // trailing 2 x 2 block [b00 b01; b10 b11] of H [y z]
    const zd b00 = A.a[3 + Q] - v1 * fy, b10 = A.a[6 + Q] - v2 * fy;
    const zd b01 = A.a[3 + R] - v1 * fz, b11 = A.a[6 + R] - v2 * fz;
    const double m = sqrt(fmax(abs2(b00) + abs2(b10), abs2(b01) + abs2(b11)));
    if (!(m > 0.0)) return 0.0;
    return sqrt(abs2(b00 * b11 - b01 * b10)) / m;
}

BEM_HD double blk_r33(const blk& A)
{
    double n0 = 0.0, n1 = 0.0, n2 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        n0 += abs2(A.a[3 * i]);
        n1 += abs2(A.a[3 * i + 1]);
        n2 += abs2(A.a[3 * i + 2]);
    }
    if (n0 >= n1 && n0 >= n2) return n0 > 0.0 ? blk_r33_piv<0>(A, sqrt(n0)) : 0.0;
    if (n1 >= n2) return blk_r33_piv<1>(A, sqrt(n1));
    return blk_r33_piv<2>(A, sqrt(n2));
}

// Smallest singular value of a 3x3 complex block: sigma_3 = |det A| / sigma_1(adj A),
// since the singular values of adj(A) are sigma_2 sigma_3, sigma_1 sigma_3, sigma_1 sigma_2.
// The rounding of det is about eps sigma_1^3, so the quotient errs by eps sigma_1^2 / sigma_2:
// on a block whose sigma_2 is small it is rounding noise far above the true sigma_3.  |r_33|
// of the pivoted QR (blk_r33) caps it there: an upper bound of sigma_3 that stays within a
// factor 3 of it and is backward stable, so the quotient stands wherever it is accurate.
BEM_HD double blk_sigma3(const blk& A)
{
    // The quotient errs by at most about eps ||A||_F^3 / |det A| relative, so |r_33| is only
    // needed where |det A| < 1e-8 ||A||_F^3; it is taken before the adjugate (A is not needed
    // after it), and tested at once
    double f2 = 0.0;
#pragma unroll
    for (int t = 0; t < 9; ++t) f2 += abs2(A.a[t]);
    const zd d0 = A.a[0] * (A.a[4] * A.a[8] - A.a[5] * A.a[7]) + A.a[1] * (A.a[5] * A.a[6] - A.a[3] * A.a[8]) +
                  A.a[2] * (A.a[3] * A.a[7] - A.a[4] * A.a[6]);
    double r33 = 1.0e300;
    if (abs2(d0) < 1e-16 * f2 * f2 * f2) r33 = blk_r33(A);
    blk adj;
    zd det = blk_det_adj(A, adj);
    double ad = sqrt(abs2(det));
    if (!(ad > 0.0) || !(r33 > 0.0)) return 0.0;
    // G = adj^H adj
    blk G;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            zd s = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) s += conj_mul(adj.a[3 * k + i], adj.a[3 * k + j]);
            G.a[3 * i + j] = s;
        }
    double l = herm3_lambda_max(G);
    if (!(l > 0.0)) return 0.0;
    return fmin(ad / sqrt(l), r33);
}

// sigma_3 of a block of any magnitude (computed on A / s, s = blk_pow2_scale(A)); the plain
// blk_sigma3 loses accuracy once the entries fall below ~1e-38 (the Gram of the adjugate
// holds eighth powers of them)
BEM_HD double blk_sigma3_scaled(const blk& A)
{
    const double sc = blk_pow2_scale(A), isc = 1.0 / sc;
    blk As;
#pragma unroll
    for (int t = 0; t < 9; ++t) As.a[t] = A.a[t] * isc;
    return sc * blk_sigma3(As);
}

// ---------------------------------------------------------------- host error plumbing

#define BEM_HIP_TRY(expr)                                  \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) {                            \
            throw bem_hip_error(e_, #expr, __FILE__, __LINE__); \
        }                                                  \
    } while (0)

#include <stdexcept>
#include <string>
struct bem_hip_error : std::runtime_error {
    hipError_t code;
    bem_hip_error(hipError_t e, const char* what, const char* file, int line)
        : std::runtime_error(std::string("HIP error ") + hipGetErrorString(e) + " in " + what + " (" + file + ":" +
                             std::to_string(line) + ")"),
          code(e)
    {
    }
};
