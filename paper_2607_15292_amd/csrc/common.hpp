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

// sigma_3 through the Householder QR with column pivoting, A P = Q R (backward stable: R is
// exact for a block within about eps ||A|| of A).  Then sigma_3 = |r_11 r_22 r_33| /
// sigma_1(adj R): the determinant is a product without cancellation, and the adjugate's
// largest singular value sigma_1 sigma_2 is dominated by its large entries, so the quotient
// is accurate down to the rounding level eps ||A|| even on blocks of numerical rank 1 or 2.
// P: the pivot column of the first step (static indices: no copies of the block, no indexed
// access); al = its norm.
template <int P>
BEM_HD double blk_sigma3_qr_piv(const blk& A, double al)
{
    constexpr int Q = P == 0 ? 1 : 0, R = P == 2 ? 1 : 2;
    // first reflection H = I - g v v^H, v = x + e^{i arg x_0} ||x|| e_0 on the pivot column x
    const zd x0 = A.a[P];
    const double a0 = sqrt(abs2(x0));
    const zd v0 = x0 + (a0 > 0.0 ? x0 * (al / a0) : zd{al, 0.0});
    const zd v1 = A.a[3 + P], v2 = A.a[6 + P];
    const double g = 2.0 / (abs2(v0) + abs2(v1) + abs2(v2));
    const zd fy = (conj_mul(v0, A.a[Q]) + conj_mul(v1, A.a[3 + Q]) + conj_mul(v2, A.a[6 + Q])) * g;
    const zd fz = (conj_mul(v0, A.a[R]) + conj_mul(v1, A.a[3 + R]) + conj_mul(v2, A.a[6 + R])) * g;
    // first row of R (|r_11| = al) and the trailing 2 x 2 block [b00 b01; b10 b11] of H [y z]
    zd r12 = A.a[Q] - v0 * fy, r13 = A.a[R] - v0 * fz;
    zd b00 = A.a[3 + Q] - v1 * fy, b10 = A.a[6 + Q] - v2 * fy;
    zd b01 = A.a[3 + R] - v1 * fz, b11 = A.a[6 + R] - v2 * fz;
    // second step: the larger column of the 2 x 2 block first
    const double ny = abs2(b00) + abs2(b10), nz = abs2(b01) + abs2(b11);
    if (nz > ny) {
        zd t = b00; b00 = b01; b01 = t;
        t = b10; b10 = b11; b11 = t;
        t = r12; r12 = r13; r13 = t;
    }
    const double a2 = sqrt(fmax(ny, nz));
    if (!(a2 > 0.0)) return 0.0;
    const double c0 = sqrt(abs2(b00));
    const zd w0 = b00 + (c0 > 0.0 ? b00 * (a2 / c0) : zd{a2, 0.0});
    const zd ph2 = c0 > 0.0 ? b00 * (-1.0 / c0) : zd{-1.0, 0.0};
    const double g2 = 2.0 / (abs2(w0) + abs2(b10));
    const zd f = (conj_mul(w0, b01) + conj_mul(b10, b11)) * g2;
    const zd r23 = b01 - w0 * f, r33 = b11 - b10 * f;
    // R = [r11 r12 r13; 0 r22 r23; 0 0 r33] with r11 = -e^{i arg x_0} al, r22 = e^{i arg b00} (-a2)
    const zd ph1 = a0 > 0.0 ? x0 * (-1.0 / a0) : zd{-1.0, 0.0};
    const zd r11 = ph1 * al, r22 = ph2 * a2;
    // adj(R), upper triangular
    blk C = blk_zero();
    C.a[0] = r22 * r33;
    C.a[1] = zd{0.0, 0.0} - r12 * r33;
    C.a[2] = r12 * r23 - r13 * r22;
    C.a[4] = r11 * r33;
    C.a[5] = zd{0.0, 0.0} - r11 * r23;
    C.a[8] = r11 * r22;
    blk G;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            zd s = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) s += conj_mul(C.a[3 * k + i], C.a[3 * k + j]);
            G.a[3 * i + j] = s;
        }
    const double l = herm3_lambda_max(G);
    if (!(l > 0.0)) return 0.0;
    return al * a2 * sqrt(abs2(r33)) / sqrt(l);
}

BEM_HD double blk_sigma3_qr(const blk& A)
{
    double n0 = 0.0, n1 = 0.0, n2 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        n0 += abs2(A.a[3 * i]);
        n1 += abs2(A.a[3 * i + 1]);
        n2 += abs2(A.a[3 * i + 2]);
    }
    if (n0 >= n1 && n0 >= n2) return n0 > 0.0 ? blk_sigma3_qr_piv<0>(A, sqrt(n0)) : 0.0;
    if (n1 >= n2) return blk_sigma3_qr_piv<1>(A, sqrt(n1));
    return blk_sigma3_qr_piv<2>(A, sqrt(n2));
}

// Smallest singular value of a 3x3 complex block: sigma_3 = |det A| / sigma_1(adj A),
// since the singular values of adj(A) are sigma_2 sigma_3, sigma_1 sigma_3, sigma_1 sigma_2.
// With determinant and adjugate from cofactors, the 2 x 2 minors err by eps sigma_1^2 and the
// quotient by about eps sigma_1^2 / sigma_2 <= eps ||A||_F^3 / |det A| relative: exact enough
// where |det A| >= 1e-8 ||A||_F^3.  Below that (blocks of numerical rank 1 or 2, where the
// quotient is rounding noise) the block goes through the pivoted QR (blk_sigma3_qr), a rare
// branch taken before the adjugate so that A is not kept live through it.
BEM_HD double blk_sigma3(const blk& A)
{
    double f2 = 0.0;
#pragma unroll
    for (int t = 0; t < 9; ++t) f2 += abs2(A.a[t]);
    const zd d0 = A.a[0] * (A.a[4] * A.a[8] - A.a[5] * A.a[7]) + A.a[1] * (A.a[5] * A.a[6] - A.a[3] * A.a[8]) +
                  A.a[2] * (A.a[3] * A.a[7] - A.a[4] * A.a[6]);
    if (abs2(d0) < 1e-16 * f2 * f2 * f2) return blk_sigma3_qr(A);
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
    return ad / sqrt(l);
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
