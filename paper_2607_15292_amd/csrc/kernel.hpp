// kernel.hpp -- Laplace-domain elastodynamic fundamental solution and collocation
// quadrature as device functions.
//
// Kernel (Appendix A, eq. (A.2) with an impulse source, Laplace transformed):
//   4 pi rho U_ij(r, s) = A(r) d_ij + B(r) rh_i rh_j,
//   A = e2/(c2^2 r) (1 + y2 + y2^2) - e1/(c1^2 r) (y1 + y1^2),
//   B = e1/(c1^2 r) (1 + 3 y1 + 3 y1^2) - e2/(c2^2 r) (1 + 3 y2 + 3 y2^2),
//   e_a = exp(-x_a), x_a = s r / c_a, y_a = 1 / x_a.
// For |x2| < 1 the 1/x^2 terms cancel; there A = e2/(c2^2 r) - I/r and
// B = 3 I/r + e1/(c1^2 r) - e2/(c2^2 r) with the lambda-integral of eq. (A.2)
//   I = int_{1/c1}^{1/c2} lam exp(-s lam r) dlam = phi(x2)/c2^2 - phi(x1)/c1^2,
//   phi(z) = sum_n (-z)^n / (n! (n + 2)).
// Traction (stress law of Sec. 2.1, t = sigma n at y, unit load in direction i at x):
//   4 pi T_ij = P1 rh_i n_j + P2 (d_ij dr/dn + rh_j n_i) + P3 rh_i rh_j dr/dn,
//   P1 = (c1^2 - 2 c2^2)(A' + B' + 2B/r) + 2 c2^2 B/r, P2 = c2^2 (A' + B/r),
//   P3 = 2 c2^2 (B' - 2B/r),  ' = d/dr.
// Quadrature per element pair (Sec. 2.3 names the Duffy transformation for the singular
// collocation integrals; rules below are the library's documented reading):
//   regular: 7-point degree-5 rule; near: the same rule on 4^m sub-triangles;
//   self: polar coordinates about the centroid on 3 sub-triangles, principal value for T
//   with the leading part g(theta)/rho^2, g = c2^2/(4 pi c1^2)(rh_i n_j - rh_j n_i),
//   integrated analytically in rho.
#pragma once

#include "common.hpp"

namespace bem {

// Element tables in mesh or cluster order, structure of arrays, FP64.
struct Geo {
    int K;
    const double *cx, *cy, *cz;     // centroid = collocation point
    const double *nx, *ny, *nz;     // unit normal
    const double *area;
    const double *lmax2;            // squared longest edge
    const double *vx, *vy, *vz;     // vertex a of element j at [a * K + j]
    const double *gx, *gy, *gz, *gw;  // regular rule points/weights (weight * area), [q * K + j]
};

template <typename T>
struct Mat {
    T c1, c2, ic1, ic2, ic1s, ic2s;  // c, 1/c, 1/c^2
    T lamc;                          // c1^2 - 2 c2^2  (lambda / rho)
    T c2s;                           // c2^2           (mu / rho)
    T inv4pirho, inv4pi;
    T gcoef;                         // c2^2 / (4 pi c1^2): leading in-plane traction
};

struct QuadTab {
    int near_on;
    double r1sq, r2sq;
    int nt, nr;
    double tx[16], tw[16], rx[16], rw[16];
    double crho;                     // sum_k w_k / (1 + x_k) of the rho rule
    double b7[21], w7[7];            // 7-point rule (barycentric, weights summing to 1)
};

// Frequencies: s_l and 1/s_l in both precisions.
struct Freq {
    int L;
    const zd *s, *sinv;
    const zf *sf, *sinvf;
};

// ---------------------------------------------------------------- math per precision

template <typename T> struct M_;

template <> struct M_<double> {
    static BEM_HD zd cexpm(zd x)  // exp(-x)
    {
        double e = exp(-x.re);
        double sn, cs;
        sincos(x.im, &sn, &cs);
        return {e * cs, -e * sn};
    }
    static BEM_HD double rsq(double a) { return 1.0 / sqrt(a); }
};

#if defined(__HIP_DEVICE_COMPILE__)
template <> struct M_<float> {
    static __device__ __forceinline__ zf cexpm(zf x)
    {
        float e = __expf(-x.re);
        float t = x.im * 0.15915494309189535f;  // revolutions
        t = t - rintf(t);
        float sn = __builtin_amdgcn_sinf(t), cs = __builtin_amdgcn_cosf(t);
        return {e * cs, -e * sn};
    }
    static __device__ __forceinline__ float rsq(float a) { return __builtin_amdgcn_rsqf(a); }
};
#else
template <> struct M_<float> {
    static inline zf cexpm(zf x)
    {
        float e = expf(-x.re);
        return {e * cosf(x.im), -e * sinf(x.im)};
    }
    static inline float rsq(float a) { return 1.0f / sqrtf(a); }
};
#endif

// Series terms: phi_n = 1/(n!(n+2)), chi_n = 1/(n!(n+3)).
template <typename T> struct Series;
template <> struct Series<double> { static constexpr int N = 20; };
template <> struct Series<float> { static constexpr int N = 11; };

constexpr double fact_inv(int n) { return n <= 1 ? 1.0 : fact_inv(n - 1) / n; }
constexpr double ser_phi(int n) { return fact_inv(n) / (n + 2); }
constexpr double ser_chi(int n) { return fact_inv(n) / (n + 3); }

#define BEM_SER21(f) {f(0), f(1), f(2), f(3), f(4), f(5), f(6), f(7), f(8), f(9), f(10), f(11), f(12), \
                      f(13), f(14), f(15), f(16), f(17), f(18), f(19), f(20)}
#define BEM_SER12(f) {(float)f(0), (float)f(1), (float)f(2), (float)f(3), (float)f(4), (float)f(5), (float)f(6), \
                      (float)f(7), (float)f(8), (float)f(9), (float)f(10), (float)f(11)}

// The coefficient tables live in constant memory and the Horner loops stay rolled, reading
// one coefficient per step: unrolled, the 20-odd FP64 literals per series are hoisted into
// registers and double the register footprint of every kernel evaluation.
#if defined(__HIP_DEVICE_COMPILE__)
static __constant__ double SER_PHI_D[21] = BEM_SER21(ser_phi);
static __constant__ double SER_CHI_D[21] = BEM_SER21(ser_chi);
static __constant__ float SER_PHI_F[12] = BEM_SER12(ser_phi);
static __constant__ float SER_CHI_F[12] = BEM_SER12(ser_chi);
template <typename T> __device__ __forceinline__ T ser_c(int n, bool chi);
template <> __device__ __forceinline__ double ser_c<double>(int n, bool chi) { return chi ? SER_CHI_D[n] : SER_PHI_D[n]; }
template <> __device__ __forceinline__ float ser_c<float>(int n, bool chi) { return chi ? SER_CHI_F[n] : SER_PHI_F[n]; }
#else
template <typename T> inline T ser_c(int n, bool chi) { return (T)(chi ? ser_chi(n) : ser_phi(n)); }
#endif

// phi(z_a) = sum (-z_a)^n phi_n and chi(z_a) = sum (-z_a)^n chi_n (a = 1, 2) by Horner in
// w = -z, both arguments in one loop.
template <typename T>
BEM_HD void phi_chi2(cx<T> z1, cx<T> z2, cx<T>& phi1, cx<T>& phi2, cx<T>& chi1, cx<T>& chi2, bool need_chi)
{
    constexpr int N = Series<T>::N;
    const cx<T> w1 = -z1, w2 = -z2;
    {
        const T c = ser_c<T>(N, false);
        cx<T> p1 = {c, (T)0}, p2 = {c, (T)0};
#pragma unroll 1
        for (int n = N - 1; n >= 0; --n) {
            const cx<T> cn = {ser_c<T>(n, false), (T)0};
            p1 = fma_c(p1, w1, cn);
            p2 = fma_c(p2, w2, cn);
        }
        phi1 = p1;
        phi2 = p2;
    }
    if (need_chi) {
        const T c = ser_c<T>(N, true);
        cx<T> q1 = {c, (T)0}, q2 = {c, (T)0};
#pragma unroll 1
        for (int n = N - 1; n >= 0; --n) {
            const cx<T> cn = {ser_c<T>(n, true), (T)0};
            q1 = fma_c(q1, w1, cn);
            q2 = fma_c(q2, w2, cn);
        }
        chi1 = q1;
        chi2 = q2;
    }
}

// A and B of 4 pi rho U = A d + B rh rh (and A', B' when DERIV).
template <typename T, bool DERIV>
BEM_HD void kernel_AB(T r, T rinv, cx<T> s, cx<T> sinv, const Mat<T>& M, cx<T>& A, cx<T>& B, cx<T>& Ad, cx<T>& Bd)
{
    const T one = (T)1;
    cx<T> x1 = s * (r * M.ic1), x2 = s * (r * M.ic2);
    cx<T> e1 = M_<T>::cexpm(x1), e2 = M_<T>::cexpm(x2);
    cx<T> e1r = e1 * (M.ic1s * rinv), e2r = e2 * (M.ic2s * rinv);
    if (abs2(x2) < one) {
        cx<T> p1, p2, q1, q2;
        phi_chi2<T>(x1, x2, p1, p2, q1, q2, DERIV);
        cx<T> Ir = (p2 * M.ic2s - p1 * M.ic1s) * rinv;  // I / r
        A = e2r - Ir;
        B = (T)3 * Ir + e1r - e2r;
        if (DERIV) {
            cx<T> Ipr = -((x2 * q2) * M.ic2s - (x1 * q1) * M.ic1s) * rinv;  // I' (dI/dr)
            cx<T> Ipr_r = Ipr * rinv, Ir_r = Ir * rinv;
            cx<T> t1 = (e1r * rinv) * (x1 + cx<T>{one, 0});
            cx<T> t2 = (e2r * rinv) * (x2 + cx<T>{one, 0});
            Ad = Ir_r - Ipr_r - t2;
            Bd = (T)3 * (Ipr_r - Ir_r) - t1 + t2;
        }
    } else {
        cx<T> y1 = sinv * (M.c1 * rinv), y2 = sinv * (M.c2 * rinv);
        cx<T> q1 = y1 + y1 * y1, q2 = y2 + y2 * y2;
        A = e2r * (q2 + cx<T>{one, 0}) - e1r * q1;
        B = e1r * ((T)3 * q1 + cx<T>{one, 0}) - e2r * ((T)3 * q2 + cx<T>{one, 0});
        if (DERIV) {
            cx<T> a1 = e1r * rinv, a2 = e2r * rinv;
            // A' = -(e2r/r)(x2 + 2 + 3 q2) + (e1r/r)(1 + 3 q1)
            Ad = a1 * ((T)3 * q1 + cx<T>{one, 0}) - a2 * (x2 + (T)3 * q2 + cx<T>{(T)2, 0});
            // B' = -(e1r/r)(x1 + 4 + 9 q1) + (e2r/r)(x2 + 4 + 9 q2)
            Bd = a2 * (x2 + (T)9 * q2 + cx<T>{(T)4, 0}) - a1 * (x1 + (T)9 * q1 + cx<T>{(T)4, 0});
        }
    }
}

// ---------------------------------------------------------------- accumulators

template <typename T>
struct AccV {
    cx<T> A, B[6];  // B: 00 01 02 11 12 22
    BEM_HD void zero()
    {
        A = {0, 0};
        for (int t = 0; t < 6; ++t) B[t] = {0, 0};
    }
    BEM_HD void add(T rx, T ry, T rz, T w, cx<T> s, cx<T> sinv, const Mat<T>& M)
    {
        T r2 = rx * rx + ry * ry + rz * rz;
        T rinv = M_<T>::rsq(r2);
        T r = r2 * rinv;
        cx<T> a, b, ad, bd;
        kernel_AB<T, false>(r, rinv, s, sinv, M, a, b, ad, bd);
        T hx = rx * rinv, hy = ry * rinv, hz = rz * rinv;
        A += w * a;
        cx<T> wb = w * b;
        B[0] += wb * (hx * hx);
        B[1] += wb * (hx * hy);
        B[2] += wb * (hx * hz);
        B[3] += wb * (hy * hy);
        B[4] += wb * (hy * hz);
        B[5] += wb * (hz * hz);
    }
    BEM_HD void store(blk& out, double scale) const
    {
        const int map[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
        for (int t = 0; t < 9; ++t) {
            zd v = cvt<double>(B[map[t]]);
            if (t == 0 || t == 4 || t == 8) v += cvt<double>(A);
            out.a[t] = v * scale;
        }
    }
};

template <typename T>
struct AccK {
    cx<T> a1[3], s2, a2[3], m3[6];
    BEM_HD void zero()
    {
        for (int t = 0; t < 3; ++t) a1[t] = a2[t] = {0, 0};
        s2 = {0, 0};
        for (int t = 0; t < 6; ++t) m3[t] = {0, 0};
    }
    BEM_HD void add(T rx, T ry, T rz, T nx, T ny, T nz, T w, cx<T> s, cx<T> sinv, const Mat<T>& M)
    {
        T h[3], rn;
        cx<T> P1, P2, P3;
        eval(rx, ry, rz, nx, ny, nz, s, sinv, M, h, rn, P1, P2, P3);
        accum(h, rn, P1, P2, P3, w);
    }
    // the traction kernel's scalars at r = y - x: rh, dr/dn and P1, P2, P3 (4 pi T =
    // P1 rh_i n_j + P2 (d_ij dr/dn + rh_j n_i) + P3 rh_i rh_j dr/dn)
    BEM_HD static void eval(T rx, T ry, T rz, T nx, T ny, T nz, cx<T> s, cx<T> sinv, const Mat<T>& M, T h[3], T& rn,
                            cx<T>& P1, cx<T>& P2, cx<T>& P3)
    {
        T r2 = rx * rx + ry * ry + rz * rz;
        T rinv = M_<T>::rsq(r2);
        T r = r2 * rinv;
        cx<T> a, b, ad, bd;
        kernel_AB<T, true>(r, rinv, s, sinv, M, a, b, ad, bd);
        h[0] = rx * rinv;
        h[1] = ry * rinv;
        h[2] = rz * rinv;
        rn = h[0] * nx + h[1] * ny + h[2] * nz;
        cx<T> br = b * rinv;
        P1 = M.lamc * (ad + bd + (T)2 * br) + ((T)2 * M.c2s) * br;
        P2 = M.c2s * (ad + br);
        P3 = ((T)2 * M.c2s) * (bd - (T)2 * br);
    }
    BEM_HD void accum(const T h[3], T rn, cx<T> P1, cx<T> P2, cx<T> P3, T w)
    {
        cx<T> wP1 = w * P1, wP2 = w * P2, wP3 = (w * rn) * P3;
        for (int t = 0; t < 3; ++t) {
            a1[t] += wP1 * h[t];
            a2[t] += wP2 * h[t];
        }
        s2 += wP2 * rn;
        m3[0] += wP3 * (h[0] * h[0]);
        m3[1] += wP3 * (h[0] * h[1]);
        m3[2] += wP3 * (h[0] * h[2]);
        m3[3] += wP3 * (h[1] * h[1]);
        m3[4] += wP3 * (h[1] * h[2]);
        m3[5] += wP3 * (h[2] * h[2]);
    }
    BEM_HD void store(blk& out, double nx, double ny, double nz, double scale) const
    {
        const int map[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
        double n[3] = {nx, ny, nz};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                zd v = cvt<double>(a1[i]) * n[j] + cvt<double>(a2[j]) * n[i] + cvt<double>(m3[map[3 * i + j]]);
                if (i == j) v += cvt<double>(s2);
                out.a[3 * i + j] = v * scale;
            }
    }
};

// ---------------------------------------------------------------- pair classes

enum { CLS_REGULAR = 0, CLS_NEAR1 = 1, CLS_NEAR2 = 2, CLS_SELF = 3 };

// Same decision, in FP64 without contraction, as the reference reading: self if i == j;
// with near_on, m = 2 if |x_i - c_j|^2 < r1^2 lmax_j^2, m = 1 if < r2^2 lmax_j^2.
BEM_HD int pair_class(const Geo& g, int i, int j, const QuadTab& Q)
{
#pragma clang fp contract(off)
    if (i == j) return CLS_SELF;
    if (!Q.near_on) return CLS_REGULAR;
    double dx = g.cx[i] - g.cx[j], dy = g.cy[i] - g.cy[j], dz = g.cz[i] - g.cz[j];
    double d2 = dx * dx + dy * dy + dz * dz;
    double l2 = g.lmax2[j];
    if (d2 < Q.r1sq * l2) return CLS_NEAR2;
    if (d2 < Q.r2sq * l2) return CLS_NEAR1;
    return CLS_REGULAR;
}

// ---------------------------------------------------------------- entries

// Regular pair in precision T (collocation point x_i, 7-point rule on element j).
template <typename T>
BEM_HD void entry_regular(const Geo& g, int op, int i, int j, cx<T> s, cx<T> sinv, const Mat<T>& M, blk& out)
{
    const int K = g.K;
    double xi = g.cx[i], yi = g.cy[i], zi = g.cz[i];
    if (op == 0) {
        AccV<T> acc;
        acc.zero();
        for (int q = 0; q < 7; ++q) {
            int o = q * K + j;
            acc.add((T)(g.gx[o] - xi), (T)(g.gy[o] - yi), (T)(g.gz[o] - zi), (T)g.gw[o], s, sinv, M);
        }
        acc.store(out, (double)M.inv4pirho);
    } else {
        AccK<T> acc;
        acc.zero();
        T nx = (T)g.nx[j], ny = (T)g.ny[j], nz = (T)g.nz[j];
        for (int q = 0; q < 7; ++q) {
            int o = q * K + j;
            acc.add((T)(g.gx[o] - xi), (T)(g.gy[o] - yi), (T)(g.gz[o] - zi), nx, ny, nz, (T)g.gw[o], s, sinv, M);
        }
        acc.store(out, g.nx[j], g.ny[j], g.nz[j], (double)M.inv4pi);
    }
}

// Units of a pair's rule: the regular rule is one unit, the near rule of level m has 4^m
// sub-triangles (7 points each), the self rule 3 nt angular lines (nr points each).  A unit
// costs about one regular entry, so entries of near and self pairs can be split over lanes.
BEM_HD int rule_units(int cls, const QuadTab& Q)
{
    return cls == CLS_SELF ? 3 * Q.nt : (cls == CLS_REGULAR ? 1 : (1 << (2 * cls)));
}

// Near pair, sub-triangle u of the 4^m congruent children (children ordered (p0,m01,m20),
// (m01,p1,m12), (m20,m12,p2), (m01,m12,m20) at every level, u read in base 4 from the top
// level); 7-point rule on it, FP64.  KOP: 0 = V, 1 = K.
template <int KOP>
BEM_HD void near_unit(const Geo& g, int i, int j, int m, int u, zd s, zd sinv, const Mat<double>& M,
                      const QuadTab& Q, blk& out)
{
    const int K = g.K;
    const double x[3] = {g.cx[i], g.cy[i], g.cz[i]};
    double P[3][3];
    for (int a = 0; a < 3; ++a) {
        P[a][0] = g.vx[a * K + j];
        P[a][1] = g.vy[a * K + j];
        P[a][2] = g.vz[a * K + j];
    }
    const double wA = g.area[j] / (double)(1 << (2 * m));
    for (int lev = m - 1; lev >= 0; --lev) {
        const int c = (u >> (2 * lev)) & 3;
        double m01[3], m12[3], m20[3];
        for (int k = 0; k < 3; ++k) {
            m01[k] = 0.5 * (P[0][k] + P[1][k]);
            m12[k] = 0.5 * (P[1][k] + P[2][k]);
            m20[k] = 0.5 * (P[2][k] + P[0][k]);
        }
        for (int k = 0; k < 3; ++k) {
            const double p0 = P[0][k], p1 = P[1][k], p2 = P[2][k];
            if (c == 0) { P[0][k] = p0;     P[1][k] = m01[k]; P[2][k] = m20[k]; }
            else if (c == 1) { P[0][k] = m01[k]; P[1][k] = p1;     P[2][k] = m12[k]; }
            else if (c == 2) { P[0][k] = m20[k]; P[1][k] = m12[k]; P[2][k] = p2; }
            else { P[0][k] = m01[k]; P[1][k] = m12[k]; P[2][k] = m20[k]; }
        }
    }
    if constexpr (KOP == 0) {
        AccV<double> acc;
        acc.zero();
#pragma unroll 1
        for (int q = 0; q < 7; ++q) {
            const double b0 = Q.b7[3 * q], b1 = Q.b7[3 * q + 1], b2 = Q.b7[3 * q + 2];
            double y[3];
            for (int k = 0; k < 3; ++k) y[k] = b0 * P[0][k] + b1 * P[1][k] + b2 * P[2][k];
            acc.add(y[0] - x[0], y[1] - x[1], y[2] - x[2], Q.w7[q] * wA, s, sinv, M);
        }
        acc.store(out, M.inv4pirho);
    } else {
        const double n[3] = {g.nx[j], g.ny[j], g.nz[j]};
        AccK<double> acc;
        acc.zero();
#pragma unroll 1
        for (int q = 0; q < 7; ++q) {
            const double b0 = Q.b7[3 * q], b1 = Q.b7[3 * q + 1], b2 = Q.b7[3 * q + 2];
            double y[3];
            for (int k = 0; k < 3; ++k) y[k] = b0 * P[0][k] + b1 * P[1][k] + b2 * P[2][k];
            acc.add(y[0] - x[0], y[1] - x[1], y[2] - x[2], n[0], n[1], n[2], Q.w7[q] * wA, s, sinv, M);
        }
        acc.store(out, n[0], n[1], n[2], M.inv4pi);
    }
}

// Self pair, angular line it of the polar rule on the sub-triangle (x, va, vb) about the
// collocation point x (the centroid), element normal n; FP64.  For T the principal value of
// the line is w_theta [sum_rho w_rho rho T + g(theta) (ln R(theta) - crho)], crho =
// sum_k w_k / rho_k being independent of R for the scaled Gauss-Legendre rule.
template <int KOP>
BEM_HD void self_line(const double x[3], const double va[3], const double vb[3], const double n[3], int it, zd s,
                      zd sinv, const Mat<double>& M, const QuadTab& Q, blk& out)
{
    double t[3] = {vb[0] - va[0], vb[1] - va[1], vb[2] - va[2]};
    const double le = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    for (int k = 0; k < 3; ++k) t[k] /= le;
    const double proj = (x[0] - va[0]) * t[0] + (x[1] - va[1]) * t[1] + (x[2] - va[2]) * t[2];
    double foot[3], p[3];
    for (int k = 0; k < 3; ++k) {
        foot[k] = va[k] + proj * t[k];
        p[k] = foot[k] - x[k];
    }
    const double d = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    for (int k = 0; k < 3; ++k) p[k] /= d;
    const double sa = (va[0] - foot[0]) * t[0] + (va[1] - foot[1]) * t[1] + (va[2] - foot[2]) * t[2];
    const double sb = (vb[0] - foot[0]) * t[0] + (vb[1] - foot[1]) * t[1] + (vb[2] - foot[2]) * t[2];
    const double ta = atan2(sa, d), tb = atan2(sb, d);
    const double hth = 0.5 * (tb - ta), mth = 0.5 * (ta + tb);
    const double th = mth + hth * Q.tx[it];
    const double wth = hth * Q.tw[it];
    double sn, cs;
    sincos(th, &sn, &cs);
    const double R = d / cs;
    const double dir[3] = {cs * p[0] + sn * t[0], cs * p[1] + sn * t[1], cs * p[2] + sn * t[2]};
    if constexpr (KOP == 0) {
        AccV<double> acc;
        acc.zero();
        for (int ir = 0; ir < Q.nr; ++ir) {
            const double rho = 0.5 * R * (1.0 + Q.rx[ir]);
            const double w = wth * (0.5 * R * Q.rw[ir]) * rho;
            acc.add(rho * dir[0], rho * dir[1], rho * dir[2], w, s, sinv, M);
        }
        acc.store(out, M.inv4pirho);
    } else {
        AccK<double> acc;
        acc.zero();
        for (int ir = 0; ir < Q.nr; ++ir) {
            const double rho = 0.5 * R * (1.0 + Q.rx[ir]);
            const double w = wth * (0.5 * R * Q.rw[ir]) * rho;
            acc.add(rho * dir[0], rho * dir[1], rho * dir[2], n[0], n[1], n[2], w, s, sinv, M);
        }
        acc.store(out, n[0], n[1], n[2], M.inv4pi);
        const double c = wth * (log(R) - Q.crho);
        for (int ii = 0; ii < 3; ++ii)
            for (int jj = 0; jj < 3; ++jj) out.a[3 * ii + jj].re += M.gcoef * c * (dir[ii] * n[jj] - dir[jj] * n[ii]);
    }
}

// Unit u = (sub-triangle a = u / nt, angle index u % nt) of element j's self rule.
template <int KOP>
BEM_HD void self_unit(const Geo& g, int j, int u, zd s, zd sinv, const Mat<double>& M, const QuadTab& Q, blk& out)
{
    const int K = g.K;
    const double x[3] = {g.cx[j], g.cy[j], g.cz[j]};
    const int a = u / Q.nt, it = u - (u / Q.nt) * Q.nt;
    const int b = (a + 1) % 3;
    const double va[3] = {g.vx[a * K + j], g.vy[a * K + j], g.vz[a * K + j]};
    const double vb[3] = {g.vx[b * K + j], g.vy[b * K + j], g.vz[b * K + j]};
    const double n[3] = {g.nx[j], g.ny[j], g.nz[j]};
    self_line<KOP>(x, va, vb, n, it, s, sinv, M, Q, out);
}

// Unit u of the rule of a near (cls 1, 2) or self (cls 3) pair.
template <int KOP>
BEM_HD void entry_unit(const Geo& g, int i, int j, int cls, int u, zd s, zd sinv, const Mat<double>& M,
                       const QuadTab& Q, blk& out)
{
    if (cls == CLS_SELF) self_unit<KOP>(g, j, u, s, sinv, M, Q, out);
    else near_unit<KOP>(g, i, j, cls, u, s, sinv, M, Q, out);
}

// Near pair (4^m sub-triangles) and self pair (polar rule): the sums of their units.
BEM_HD void entry_near(const Geo& g, int op, int i, int j, int m, zd s, zd sinv, const Mat<double>& M,
                       const QuadTab& Q, blk& out)
{
    out = blk_zero();
    const int nu = 1 << (2 * m);
    for (int u = 0; u < nu; ++u) {
        blk e;
        if (op == 0) near_unit<0>(g, i, j, m, u, s, sinv, M, Q, e);
        else near_unit<1>(g, i, j, m, u, s, sinv, M, Q, e);
        for (int t = 0; t < 9; ++t) out.a[t] += e.a[t];
    }
}

BEM_HD void entry_self(const Geo& g, int op, int j, zd s, zd sinv, const Mat<double>& M, const QuadTab& Q,
                       blk& out)
{
    out = blk_zero();
    const int nu = 3 * Q.nt;
    for (int u = 0; u < nu; ++u) {
        blk e;
        if (op == 0) self_unit<0>(g, j, u, s, sinv, M, Q, e);
        else self_unit<1>(g, j, u, s, sinv, M, Q, e);
        for (int t = 0; t < 9; ++t) out.a[t] += e.a[t];
    }
}

// ---------------------------------------------------------------- double layer, linear basis

// Barycentric coordinate of vertex v of element j at a point y of its plane (the hat function
// of eqs. (subspace), (basis) of the vertex's node restricted to the element):
// lambda_v(y) = n . ((P_{v+1} - y) x (P_{v+2} - y)) / (2 A).
BEM_HD double bary_at(const Geo& g, int j, int v, const double y[3])
{
    const int K = g.K, a = (v + 1) % 3, b = (v + 2) % 3;
    const double p[3] = {g.vx[a * K + j] - y[0], g.vy[a * K + j] - y[1], g.vz[a * K + j] - y[2]};
    const double q[3] = {g.vx[b * K + j] - y[0], g.vy[b * K + j] - y[1], g.vz[b * K + j] - y[2]};
    const double cr[3] = {p[1] * q[2] - p[2] * q[1], p[2] * q[0] - p[0] * q[2], p[0] * q[1] - p[1] * q[0]};
    return (g.nx[j] * cr[0] + g.ny[j] * cr[1] + g.nz[j] * cr[2]) / (2.0 * g.area[j]);
}

// The double layer of pair (i, j) against the three hat functions of element j's vertices:
// out[v] = int_{gamma_j} T(x_i, y) lambda_v(y) dy, each kernel evaluation shared by the three
// weights, with the rule of the pair's class (FP64).  Self pair: the principal value of the
// leading part g(theta) / rho^2 is taken with the weight lambda_v(x_i) = 1/3; the remainder
// T (lambda_v(y) - 1/3) is weakly singular and integrated by the polar rule.
BEM_HD void entry_kl3(const Geo& g, int i, int j, zd s, zd sinv, const Mat<double>& M, const QuadTab& Q, blk out[3])
{
    const int K = g.K;
    const int cls = pair_class(g, i, j, Q);
    const double x[3] = {g.cx[i], g.cy[i], g.cz[i]};
    const double n[3] = {g.nx[j], g.ny[j], g.nz[j]};
    AccK<double> acc[3];
    for (int v = 0; v < 3; ++v) acc[v].zero();
    auto point = [&](const double y[3], double w, const double lw[3]) {
        double h[3], rn;
        zd P1, P2, P3;
        AccK<double>::eval(y[0] - x[0], y[1] - x[1], y[2] - x[2], n[0], n[1], n[2], s, sinv, M, h, rn, P1, P2, P3);
        for (int v = 0; v < 3; ++v) acc[v].accum(h, rn, P1, P2, P3, w * lw[v]);
    };
    for (int v = 0; v < 3; ++v) out[v] = blk_zero();
    if (cls == CLS_REGULAR) {
        for (int q = 0; q < 7; ++q) {
            const int o = q * K + j;
            const double y[3] = {g.gx[o], g.gy[o], g.gz[o]};
            const double lw[3] = {Q.b7[3 * q], Q.b7[3 * q + 1], Q.b7[3 * q + 2]};
            point(y, g.gw[o], lw);
        }
    } else if (cls != CLS_SELF) {
        const int m = cls, nu = 1 << (2 * m);
        const double wA = g.area[j] / (double)nu;
        for (int u = 0; u < nu; ++u) {
            double P[3][3];
            for (int a = 0; a < 3; ++a) {
                P[a][0] = g.vx[a * K + j];
                P[a][1] = g.vy[a * K + j];
                P[a][2] = g.vz[a * K + j];
            }
            for (int lev = m - 1; lev >= 0; --lev) {
                const int c = (u >> (2 * lev)) & 3;
                double m01[3], m12[3], m20[3];
                for (int k = 0; k < 3; ++k) {
                    m01[k] = 0.5 * (P[0][k] + P[1][k]);
                    m12[k] = 0.5 * (P[1][k] + P[2][k]);
                    m20[k] = 0.5 * (P[2][k] + P[0][k]);
                }
                for (int k = 0; k < 3; ++k) {
                    const double p0 = P[0][k], p1 = P[1][k], p2 = P[2][k];
                    if (c == 0) { P[0][k] = p0;     P[1][k] = m01[k]; P[2][k] = m20[k]; }
                    else if (c == 1) { P[0][k] = m01[k]; P[1][k] = p1;     P[2][k] = m12[k]; }
                    else if (c == 2) { P[0][k] = m20[k]; P[1][k] = m12[k]; P[2][k] = p2; }
                    else { P[0][k] = m01[k]; P[1][k] = m12[k]; P[2][k] = m20[k]; }
                }
            }
            for (int q = 0; q < 7; ++q) {
                const double b0 = Q.b7[3 * q], b1 = Q.b7[3 * q + 1], b2 = Q.b7[3 * q + 2];
                double y[3];
                for (int k = 0; k < 3; ++k) y[k] = b0 * P[0][k] + b1 * P[1][k] + b2 * P[2][k];
                const double lw[3] = {bary_at(g, j, 0, y), bary_at(g, j, 1, y), bary_at(g, j, 2, y)};
                point(y, Q.w7[q] * wA, lw);
            }
        }
    } else {
        const double lx[3] = {bary_at(g, j, 0, x), bary_at(g, j, 1, x), bary_at(g, j, 2, x)};
        for (int a = 0; a < 3; ++a) {
            const int b = (a + 1) % 3;
            const double va[3] = {g.vx[a * K + j], g.vy[a * K + j], g.vz[a * K + j]};
            const double vb[3] = {g.vx[b * K + j], g.vy[b * K + j], g.vz[b * K + j]};
            double t[3] = {vb[0] - va[0], vb[1] - va[1], vb[2] - va[2]};
            const double le = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
            for (int k = 0; k < 3; ++k) t[k] /= le;
            const double proj = (x[0] - va[0]) * t[0] + (x[1] - va[1]) * t[1] + (x[2] - va[2]) * t[2];
            double foot[3], p[3];
            for (int k = 0; k < 3; ++k) {
                foot[k] = va[k] + proj * t[k];
                p[k] = foot[k] - x[k];
            }
            const double d = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
            for (int k = 0; k < 3; ++k) p[k] /= d;
            const double sa = (va[0] - foot[0]) * t[0] + (va[1] - foot[1]) * t[1] + (va[2] - foot[2]) * t[2];
            const double sb = (vb[0] - foot[0]) * t[0] + (vb[1] - foot[1]) * t[1] + (vb[2] - foot[2]) * t[2];
            const double ta = atan2(sa, d), tb = atan2(sb, d);
            const double hth = 0.5 * (tb - ta), mth = 0.5 * (ta + tb);
            for (int it = 0; it < Q.nt; ++it) {
                const double th = mth + hth * Q.tx[it];
                const double wth = hth * Q.tw[it];
                double sn, cs;
                sincos(th, &sn, &cs);
                const double R = d / cs;
                const double dir[3] = {cs * p[0] + sn * t[0], cs * p[1] + sn * t[1], cs * p[2] + sn * t[2]};
                for (int ir = 0; ir < Q.nr; ++ir) {
                    const double rho = 0.5 * R * (1.0 + Q.rx[ir]);
                    const double y[3] = {x[0] + rho * dir[0], x[1] + rho * dir[1], x[2] + rho * dir[2]};
                    const double lw[3] = {bary_at(g, j, 0, y), bary_at(g, j, 1, y), bary_at(g, j, 2, y)};
                    point(y, wth * (0.5 * R * Q.rw[ir]) * rho, lw);
                }
                const double c = wth * (log(R) - Q.crho);
                for (int ii = 0; ii < 3; ++ii)
                    for (int jj = 0; jj < 3; ++jj) {
                        const double gv = M.gcoef * c * (dir[ii] * n[jj] - dir[jj] * n[ii]);
                        for (int v = 0; v < 3; ++v) out[v].a[3 * ii + jj].re += lx[v] * gv;
                    }
            }
        }
    }
    for (int v = 0; v < 3; ++v) {
        blk e;
        acc[v].store(e, n[0], n[1], n[2], M.inv4pi);
        for (int q = 0; q < 9; ++q) out[v].a[q] += e.a[q];
    }
}

}  // namespace bem
