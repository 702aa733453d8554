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
BEM_HD double blk_r33(const blk& A)
{
    double n[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i) n[j] += abs2(A.a[3 * i + j]);
    const int p = n[0] >= n[1] ? (n[0] >= n[2] ? 0 : 2) : (n[1] >= n[2] ? 1 : 2);
    const double al = sqrt(n[p]);
    if (!(al > 0.0)) return 0.0;
    // v = x + e^{i arg x_0} ||x|| e_0, H = I - 2 v v^H / (v^H v)
    zd v[3] = {A.a[p], A.a[3 + p], A.a[6 + p]};
    const double a0 = sqrt(abs2(v[0]));
    const zd ph = a0 > 0.0 ? v[0] * (1.0 / a0) : zd{1.0, 0.0};
    v[0] += ph * al;
    const double vv = abs2(v[0]) + abs2(v[1]) + abs2(v[2]);
    zd B[2][2];
    int c = 0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        if (q == p) continue;
        const zd y[3] = {A.a[q], A.a[3 + q], A.a[6 + q]};
        const zd w = conj_mul(v[0], y[0]) + conj_mul(v[1], y[1]) + conj_mul(v[2], y[2]);
        const zd f = w * (2.0 / vv);
        B[0][c] = y[1] - v[1] * f;
        B[1][c] = y[2] - v[2] * f;
        ++c;
    }
    const double m = sqrt(fmax(abs2(B[0][0]) + abs2(B[1][0]), abs2(B[0][1]) + abs2(B[1][1])));
    if (!(m > 0.0)) return 0.0;
    const zd det = B[0][0] * B[1][1] - B[0][1] * B[1][0];
    return sqrt(abs2(det)) / m;
}

// Smallest singular value of a 3x3 complex block: sigma_3 = |det A| / sigma_1(adj A),
// since the singular values of adj(A) are sigma_2 sigma_3, sigma_1 sigma_3, sigma_1 sigma_2.
// The rounding of det is about eps sigma_1^3, so the quotient errs by eps sigma_1^2 / sigma_2:
// on a block whose sigma_2 is small it is rounding noise far above the true sigma_3.  Two
// upper bounds of sigma_3 that stay accurate there cap it: |r_33| of the pivoted QR
// (blk_r33) and sigma_2 <= sqrt(3) sigma_1(adj A) / ||A||_F; neither is below sigma_3, so the
// quotient stands wherever it is accurate (a well-conditioned block).
BEM_HD double blk_sigma3(const blk& A)
{
    blk adj;
    zd det = blk_det_adj(A, adj);
    double ad = sqrt(abs2(det));
    if (!(ad > 0.0)) return 0.0;
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
    const double sa = sqrt(l);
    double f2 = 0.0;
#pragma unroll
    for (int t = 0; t < 9; ++t) f2 += abs2(A.a[t]);
    return fmin(fmin(ad / sa, 1.7320508075688772 * sa / sqrt(f2)), blk_r33(A));
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
