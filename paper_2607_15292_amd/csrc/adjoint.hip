// adjoint.hip -- matrix-free products with the dense discrete operator (entries recomputed,
// never stored) and the adjoint of the single layer: the gradient of the bilinear form
// Re S, S = sum_{r, l} w[r][l]^T V(s_l) x[r][l], with respect to the node coordinates and
// the material (the discrete operator of eq. (discrVK) at the contour points of Sec. 2.4,
// differentiated; the paper itself has no adjoint).
//
// Regular pairs: chain rule.  With r = y - x, R = |r|, rh = r / R and 4 pi rho U = A I +
// B rh rh^T, f = w^T U v has the gradient
//   grad_r f = (A' (w.v) + B' (w.rh)(v.rh)) rh + (B / R) ((v.rh) w + (w.rh) v - 2 (w.rh)(v.rh) rh),
// taken at the Gauss points y_q = sum_a b_qa P_a of element j (rows of node a; for a near
// pair, the points of the 4^m sub-triangles in barycentric coordinates of element j), minus
// at the centroid of element i, and the area of element j enters through dA/dP.  The speeds enter
// through A and B only: dA/dc1 = -e1r / c1, dA/dc2 = e2r (x2 - 1) / c2, dB/dc1 =
// e1r (x1 + 1) / c1, dB/dc2 = -e2r (x2 + 1) / c2 with x_a = s R / c_a, e_ar = exp(-x_a) /
// (c_a^2 R) (both branches of the kernel: in the series branch the lambda-integral
// contributes -+ e_a / c_a^3).  Self pairs: the derivative of the integral by the polar rule (below).
#include "lib.hpp"

namespace bem {

namespace {

constexpr int WG = 256;
constexpr int JB = 32;     // column elements per workgroup of the adjoint kernel
constexpr int NR = 4;      // right-hand sides per pass of the matrix-free product

__device__ __forceinline__ double wsum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// y[r][l][3 e + a] = sum_o ENTRY(e, o, l)[a][b] x[r][l][3 o + b]  (TRANS: ENTRY(o, e, l)[b][a]);
// thread per (e, l), e fastest; right-hand sides in passes of NR.  Two waves per SIMD (at the
// price of some spills) run it 28 % faster than the one the compiler picks by itself.
template <bool TRANS>
__global__ __launch_bounds__(WG, 2) void k_mf_apply(DevCtx c, int op, int nrhs, const zd* __restrict__ x,
                                                 zd* __restrict__ y)
{
    const int K = c.geo.K, L = c.fr.L;
    const int e = blockIdx.x * WG + threadIdx.x, l = blockIdx.y;
    if (e >= K) return;
    const size_t M = 3 * (size_t)K;
    for (int r0 = 0; r0 < nrhs; r0 += NR) {
        const int nr = min(NR, nrhs - r0);
        zd acc[NR][3];
#pragma unroll
        for (int rr = 0; rr < NR; ++rr)
#pragma unroll
            for (int a = 0; a < 3; ++a) acc[rr][a] = {0.0, 0.0};
        for (int o = 0; o < K; ++o) {
            const blk E = TRANS ? entry_dispatch<false>(c, op, o, e, l) : entry_dispatch<false>(c, op, e, o, l);
#pragma unroll
            for (int rr = 0; rr < NR; ++rr) {
                if (rr >= nr) break;
                const zd* xv = x + ((size_t)(r0 + rr) * L + l) * M + 3 * (size_t)o;
                const zd v[3] = {xv[0], xv[1], xv[2]};
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b)
                        acc[rr][a] = TRANS ? fma_c(E.a[3 * b + a], v[b], acc[rr][a]) : fma_c(E.a[3 * a + b], v[b], acc[rr][a]);
            }
        }
        for (int rr = 0; rr < nr; ++rr) {
            zd* yv = y + ((size_t)(r0 + rr) * L + l) * M + 3 * (size_t)e;
#pragma unroll
            for (int a = 0; a < 3; ++a) yv[a] = acc[rr][a];
        }
    }
}

// y[r][l][3 e + a] = sum_j sum_v (KL_v(e, j, l) g[r][l][node(j, v)])_a, plus the free term
// 1/2 * 1/3 sum_v g[r][l][node(e, v)]; thread per (e, l), e fastest; right-hand sides in
// passes of NR.  The three vertex weights of a pair share its kernel evaluations.
__global__ __launch_bounds__(WG) void k_mf_apply_kl(DevCtx c, const int* __restrict__ tri, int nnodes, int nrhs,
                                                    const zd* __restrict__ g, zd* __restrict__ y, int free_term)
{
    const int K = c.geo.K, L = c.fr.L;
    const int e = blockIdx.x * WG + threadIdx.x, l = blockIdx.y;
    if (e >= K) return;
    const size_t M = 3 * (size_t)K, N = 3 * (size_t)nnodes;
    for (int r0 = 0; r0 < nrhs; r0 += NR) {
        const int nr = min(NR, nrhs - r0);
        zd acc[NR][3];
#pragma unroll
        for (int rr = 0; rr < NR; ++rr)
#pragma unroll
            for (int a = 0; a < 3; ++a) acc[rr][a] = {0.0, 0.0};
        for (int o = 0; o < K; ++o) {
            blk E[3];
            entry_kl3(c.geo, e, o, c.fr.s[l], c.fr.sinv[l], c.md, c.qt, E);
            for (int v = 0; v < 3; ++v) {
                const int nd = tri[3 * o + v];
#pragma unroll
                for (int rr = 0; rr < NR; ++rr) {
                    if (rr >= nr) break;
                    const zd* gv = g + ((size_t)(r0 + rr) * L + l) * N + 3 * (size_t)nd;
                    const zd u[3] = {gv[0], gv[1], gv[2]};
#pragma unroll
                    for (int a = 0; a < 3; ++a)
#pragma unroll
                        for (int b = 0; b < 3; ++b) acc[rr][a] = fma_c(E[v].a[3 * a + b], u[b], acc[rr][a]);
                }
            }
        }
        for (int rr = 0; rr < nr; ++rr) {
            if (free_term)
                for (int v = 0; v < 3; ++v) {
                    const zd* gv = g + ((size_t)(r0 + rr) * L + l) * N + 3 * (size_t)tri[3 * e + v];
                    for (int a = 0; a < 3; ++a) acc[rr][a] += gv[a] * (0.5 / 3.0);
                }
            zd* yv = y + ((size_t)(r0 + rr) * L + l) * M + 3 * (size_t)e;
#pragma unroll
            for (int a = 0; a < 3; ++a) yv[a] = acc[rr][a];
        }
    }
}

// A, B, dA/dR, dB/dR and the speed derivatives of A and B at distance R.
__device__ __forceinline__ void kernel_adj(double R, double Rinv, zd s, zd sinv, const Mat<double>& M, zd& A, zd& B,
                                           zd& Ad, zd& Bd, zd& A1, zd& A2, zd& B1, zd& B2)
{
    kernel_AB<double, true>(R, Rinv, s, sinv, M, A, B, Ad, Bd);
    const zd x1 = s * (R * M.ic1), x2 = s * (R * M.ic2);
    const zd e1r = M_<double>::cexpm(x1) * (M.ic1s * Rinv), e2r = M_<double>::cexpm(x2) * (M.ic2s * Rinv);
    const zd one = {1.0, 0.0};
    A1 = e1r * (-M.ic1);
    A2 = (e2r * (x2 - one)) * M.ic2;
    B1 = (e1r * (x1 + one)) * M.ic1;
    B2 = (e2r * (x2 + one)) * (-M.ic2);
}

// Regular and near pairs (i != j; pair classes held fixed, the Gauss points of the near
// rule's sub-triangles move with the vertices): one thread per row element i, JB column
// elements per workgroup.  gJ[bx][j][3 a + k]: d Re S / dP_{j,a,k} summed over the workgroup's rows;
// gI[by][i][k]: d Re S / d(centroid of i)_k over the workgroup's columns; gM[tile]: dc1, dc2,
// Re S, Im S.
__global__ __launch_bounds__(WG) void k_adjoint_v(DevCtx c, int nrhs, const zd* __restrict__ w,
                                                  const zd* __restrict__ x, double* __restrict__ gJ,
                                                  double* __restrict__ gI, double* __restrict__ gM)
{
    __shared__ double red[WG / 64][9];
    const Geo& g = c.geo;
    const int K = g.K, L = c.fr.L;
    const size_t M = 3 * (size_t)K;
    const int i = blockIdx.x * WG + threadIdx.x;
    const bool act = i < K;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int j0 = blockIdx.y * JB, j1 = min(K, j0 + JB);
    const double pref = c.md.inv4pirho;
    double ci[3] = {0.0, 0.0, 0.0}, mat[4] = {0.0, 0.0, 0.0, 0.0};
    const double xi[3] = {act ? g.cx[i] : 0.0, act ? g.cy[i] : 0.0, act ? g.cz[i] : 0.0};
    for (int j = j0; j < j1; ++j) {
        double gj[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) gj[t] = 0.0;
        if (act && i != j) {
            // dA/dP_a of element j: dA/dP1 = (e2 x n) / 2, dA/dP2 = (n x e1) / 2, dA/dP0 = -(sum)
            double P[3][3];
            for (int a = 0; a < 3; ++a) {
                P[a][0] = g.vx[a * K + j];
                P[a][1] = g.vy[a * K + j];
                P[a][2] = g.vz[a * K + j];
            }
            const double n[3] = {g.nx[j], g.ny[j], g.nz[j]};
            const double e1[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
            const double e2[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
            double dA[3][3];
            dA[1][0] = 0.5 * (e2[1] * n[2] - e2[2] * n[1]);
            dA[1][1] = 0.5 * (e2[2] * n[0] - e2[0] * n[2]);
            dA[1][2] = 0.5 * (e2[0] * n[1] - e2[1] * n[0]);
            dA[2][0] = 0.5 * (n[1] * e1[2] - n[2] * e1[1]);
            dA[2][1] = 0.5 * (n[2] * e1[0] - n[0] * e1[2]);
            dA[2][2] = 0.5 * (n[0] * e1[1] - n[1] * e1[0]);
            for (int k = 0; k < 3; ++k) dA[0][k] = -(dA[1][k] + dA[2][k]);
            // regular pair: one unit; near pair of level m: the 4^m sub-triangles, ordered as
            // in the forward near rule; Sb[b][a] is coordinate a of sub-vertex b in P
            const int m = pair_class(g, i, j, c.qt);
            const int nsub = 1 << (2 * m);
            const double wsub = g.area[j] * pref / (double)nsub;
#pragma unroll 1
            for (int u = 0; u < nsub; ++u) {
            double Sb[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
#pragma unroll 1
            for (int lev = m - 1; lev >= 0; --lev) {
                const int ch = (u >> (2 * lev)) & 3;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double p0 = Sb[0][a], p1 = Sb[1][a], p2 = Sb[2][a];
                    const double m01 = 0.5 * (p0 + p1), m12 = 0.5 * (p1 + p2), m20 = 0.5 * (p2 + p0);
                    if (ch == 0) { Sb[1][a] = m01; Sb[2][a] = m20; }
                    else if (ch == 1) { Sb[0][a] = m01; Sb[2][a] = m12; }
                    else if (ch == 2) { Sb[0][a] = m20; Sb[1][a] = m12; }
                    else { Sb[0][a] = m01; Sb[1][a] = m12; Sb[2][a] = m20; }
                }
            }
#pragma unroll 1
            for (int q = 0; q < 7; ++q) {
                const double* bq = c.qt.b7 + 3 * q;
                double b[3], y[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) b[a] = bq[0] * Sb[0][a] + bq[1] * Sb[1][a] + bq[2] * Sb[2][a];
#pragma unroll
                for (int k = 0; k < 3; ++k) y[k] = b[0] * P[0][k] + b[1] * P[1][k] + b[2] * P[2][k];
                const double r[3] = {y[0] - xi[0], y[1] - xi[1], y[2] - xi[2]};
                const double R2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                const double Rinv = 1.0 / sqrt(R2), R = R2 * Rinv;
                const double rh[3] = {r[0] * Rinv, r[1] * Rinv, r[2] * Rinv};
                double G[3] = {0.0, 0.0, 0.0}, V = 0.0, Vi = 0.0, m1 = 0.0, m2 = 0.0;
#pragma unroll 1
                for (int l = 0; l < L; ++l) {
                    zd A, B, Ad, Bd, A1, A2, B1, B2;
                    kernel_adj(R, Rinv, c.fr.s[l], c.fr.sinv[l], c.md, A, B, Ad, Bd, A1, A2, B1, B2);
                    const zd BR = B * Rinv;
#pragma unroll 1
                    for (int rr = 0; rr < nrhs; ++rr) {
                        const zd* up = w + ((size_t)rr * L + l) * M + 3 * (size_t)i;
                        const zd* vp = x + ((size_t)rr * L + l) * M + 3 * (size_t)j;
                        const zd u[3] = {up[0], up[1], up[2]}, v[3] = {vp[0], vp[1], vp[2]};
                        const zd uv = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
                        const zd ur = u[0] * rh[0] + u[1] * rh[1] + u[2] * rh[2];
                        const zd vr = v[0] * rh[0] + v[1] * rh[1] + v[2] * rh[2];
                        const zd t2 = ur * vr;
                        const zd val = A * uv + B * t2;
                        const double gs = (Ad * uv + Bd * t2).re;
#pragma unroll
                        for (int k = 0; k < 3; ++k) G[k] += gs * rh[k] + (BR * (vr * u[k] + ur * v[k] - t2 * (2.0 * rh[k]))).re;
                        V += val.re;
                        Vi += val.im;
                        m1 += (A1 * uv + B1 * t2).re;
                        m2 += (A2 * uv + B2 * t2).re;
                    }
                }
                const double w7 = c.qt.w7[q] * pref / (double)nsub, wA = c.qt.w7[q] * wsub;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double gk = wA * G[k];
                    ci[k] -= gk;
#pragma unroll
                    for (int a = 0; a < 3; ++a) gj[3 * a + k] += b[a] * gk + w7 * V * dA[a][k];
                }
                mat[0] += wA * m1;
                mat[1] += wA * m2;
                mat[2] += wA * V;
                mat[3] += wA * Vi;
            }
            }
        }
        // sum over the workgroup's rows, in a fixed order
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const double sv = wsum(gj[t]);
            if (lane == 0) red[wv][t] = sv;
        }
        __syncthreads();
        if (threadIdx.x < 9) {
            double sv = 0.0;
            for (int q = 0; q < WG / 64; ++q) sv += red[q][threadIdx.x];
            gJ[((size_t)blockIdx.x * K + j) * 9 + threadIdx.x] = sv;
        }
        __syncthreads();
    }
    if (act)
        for (int k = 0; k < 3; ++k) gI[((size_t)blockIdx.y * K + i) * 3 + k] = ci[k];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const double sv = wsum(mat[t]);
        if (lane == 0) red[wv][t] = sv;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double sv = 0.0;
        for (int q = 0; q < WG / 64; ++q) sv += red[q][threadIdx.x];
        gM[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 4 + threadIdx.x] = sv;
    }
}

// Self pairs: the derivative of the integral, taken by hand.  With y = sum_a lambda_a(y) P_a on
// the element (barycentric coordinates fixed under a perturbation of the vertices) and the
// collocation point x = (P_0 + P_1 + P_2) / 3, the self entry is E = int U(y - x) dy and
//   dE/dP_a = int grad_r U(y - x) (lambda_a(y) - 1/3) dy + (dA/dP_a / A) E,
// whose first integrand is O(1/|y - x|) (lambda_a - 1/3 vanishes at the centroid); dE/dc =
// int dU/dc dy.  Both are integrated by the polar rule of the forward self entry.  Thread per
// element j; out[j][13]: 9 vertex derivatives (vertex a, coordinate k at 3 a + k) of Re of the
// self terms of S, their c1 and c2 derivatives, Re and Im.
__global__ __launch_bounds__(64) void k_adjoint_self(DevCtx c, int nrhs, const zd* __restrict__ w,
                                                     const zd* __restrict__ x, double* __restrict__ out)
{
    const Geo& g = c.geo;
    const QuadTab& Q = c.qt;
    const int K = g.K, L = c.fr.L;
    const size_t M = 3 * (size_t)K;
    const int j = blockIdx.x * 64 + threadIdx.x;
    if (j >= K) return;
    const double pref = c.md.inv4pirho;
    double P[3][3];
    for (int a = 0; a < 3; ++a) {
        P[a][0] = g.vx[a * K + j];
        P[a][1] = g.vy[a * K + j];
        P[a][2] = g.vz[a * K + j];
    }
    const double xc[3] = {g.cx[j], g.cy[j], g.cz[j]};
    const double n[3] = {g.nx[j], g.ny[j], g.nz[j]};
    const double e1[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
    const double e2[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
    double dA[3][3];
    dA[1][0] = 0.5 * (e2[1] * n[2] - e2[2] * n[1]);
    dA[1][1] = 0.5 * (e2[2] * n[0] - e2[0] * n[2]);
    dA[1][2] = 0.5 * (e2[0] * n[1] - e2[1] * n[0]);
    dA[2][0] = 0.5 * (n[1] * e1[2] - n[2] * e1[1]);
    dA[2][1] = 0.5 * (n[2] * e1[0] - n[0] * e1[2]);
    dA[2][2] = 0.5 * (n[0] * e1[1] - n[1] * e1[0]);
    for (int k = 0; k < 3; ++k) dA[0][k] = -(dA[1][k] + dA[2][k]);
    double gP[9], V = 0.0, Vi = 0.0, m1 = 0.0, m2 = 0.0;
    for (int t = 0; t < 9; ++t) gP[t] = 0.0;
#pragma unroll 1
    for (int sa = 0; sa < 3; ++sa) {
        const int sb = (sa + 1) % 3;
        double t[3] = {P[sb][0] - P[sa][0], P[sb][1] - P[sa][1], P[sb][2] - P[sa][2]};
        const double le = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
        for (int k = 0; k < 3; ++k) t[k] /= le;
        const double proj = (xc[0] - P[sa][0]) * t[0] + (xc[1] - P[sa][1]) * t[1] + (xc[2] - P[sa][2]) * t[2];
        double foot[3], p[3];
        for (int k = 0; k < 3; ++k) {
            foot[k] = P[sa][k] + proj * t[k];
            p[k] = foot[k] - xc[k];
        }
        const double d = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
        for (int k = 0; k < 3; ++k) p[k] /= d;
        const double qa = (P[sa][0] - foot[0]) * t[0] + (P[sa][1] - foot[1]) * t[1] + (P[sa][2] - foot[2]) * t[2];
        const double qb = (P[sb][0] - foot[0]) * t[0] + (P[sb][1] - foot[1]) * t[1] + (P[sb][2] - foot[2]) * t[2];
        const double ta = atan2(qa, d), tb = atan2(qb, d);
        const double hth = 0.5 * (tb - ta), mth = 0.5 * (ta + tb);
#pragma unroll 1
        for (int it = 0; it < Q.nt; ++it) {
            const double th = mth + hth * Q.tx[it];
            const double wth = hth * Q.tw[it];
            double sn, cs;
            sincos(th, &sn, &cs);
            const double Rl = d / cs;
            const double rh[3] = {cs * p[0] + sn * t[0], cs * p[1] + sn * t[1], cs * p[2] + sn * t[2]};
#pragma unroll 1
            for (int ir = 0; ir < Q.nr; ++ir) {
                const double rho = 0.5 * Rl * (1.0 + Q.rx[ir]);
                const double wq = wth * (0.5 * Rl * Q.rw[ir]) * rho * pref;
                const double y[3] = {xc[0] + rho * rh[0], xc[1] + rho * rh[1], xc[2] + rho * rh[2]};
                double lam[3];
                for (int a = 0; a < 3; ++a) lam[a] = bary_at(g, j, a, y) - 1.0 / 3.0;
                double G[3] = {0.0, 0.0, 0.0}, v0 = 0.0, v1 = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll 1
                for (int l = 0; l < L; ++l) {
                    zd A, B, Ad, Bd, A1, A2, B1, B2;
                    kernel_adj(rho, 1.0 / rho, c.fr.s[l], c.fr.sinv[l], c.md, A, B, Ad, Bd, A1, A2, B1, B2);
                    const zd BR = B * (1.0 / rho);
#pragma unroll 1
                    for (int rr = 0; rr < nrhs; ++rr) {
                        const zd* up = w + ((size_t)rr * L + l) * M + 3 * (size_t)j;
                        const zd* vp = x + ((size_t)rr * L + l) * M + 3 * (size_t)j;
                        const zd u[3] = {up[0], up[1], up[2]}, v[3] = {vp[0], vp[1], vp[2]};
                        const zd uv = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
                        const zd ur = u[0] * rh[0] + u[1] * rh[1] + u[2] * rh[2];
                        const zd vr = v[0] * rh[0] + v[1] * rh[1] + v[2] * rh[2];
                        const zd t2 = ur * vr;
                        const zd val = A * uv + B * t2;
                        const double gs = (Ad * uv + Bd * t2).re;
#pragma unroll
                        for (int k = 0; k < 3; ++k)
                            G[k] += gs * rh[k] + (BR * (vr * u[k] + ur * v[k] - t2 * (2.0 * rh[k]))).re;
                        v0 += val.re;
                        v1 += val.im;
                        d1 += (A1 * uv + B1 * t2).re;
                        d2 += (A2 * uv + B2 * t2).re;
                    }
                }
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int k = 0; k < 3; ++k) gP[3 * a + k] += wq * G[k] * lam[a];
                V += wq * v0;
                Vi += wq * v1;
                m1 += wq * d1;
                m2 += wq * d2;
            }
        }
    }
    double* o = out + (size_t)j * 13;
    const double ia = 1.0 / g.area[j];
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) o[3 * a + k] = gP[3 * a + k] + V * dA[a][k] * ia;
    o[9] = m1;
    o[10] = m2;
    o[11] = V;
    o[12] = Vi;
}

// ---------------------------------------------------------------- double layer

// psi(z) = sum_n (n - 1)(n - 2) (-z)^n / (n! (n + 2)) for both waves: the second derivative of
// the series part I / r of A and B is (psi(x2) / c2^2 - psi(x1) / c1^2) / r^3.
BEM_HD void psi2(zd x1, zd x2, zd& p1, zd& p2)
{
    constexpr int N = Series<double>::N;
    const zd w1 = -x1, w2 = -x2;
    const double cN = (double)((N - 1) * (N - 2)) * ser_c<double>(N, false);
    zd a = {cN, 0.0}, b = {cN, 0.0};
#pragma unroll 1
    for (int n = N - 1; n >= 0; --n) {
        const zd cn = {(double)((n - 1) * (n - 2)) * ser_c<double>(n, false), 0.0};
        a = fma_c(a, w1, cn);
        b = fma_c(b, w2, cn);
    }
    p1 = a;
    p2 = b;
}

// The traction kernel's scalars and their derivatives at distance R: P1, P2, P3 of 4 pi T =
// P1 rh n^T + P2 (dr/dn I + n rh^T) + P3 dr/dn rh rh^T, their R-derivatives and their c1 and
// c2 derivatives.  With u = 1/R, x_a = s R / c_a, e_ar = exp(-x_a) / (c_a^2 R), q_a = y_a +
// y_a^2, y_a = 1 / x_a:
//   A'' = u^2 (e2r (x2^2 + 3 x2 + 7 + 12 q2) - e1r (x1 + 5 + 12 q1)),
//   B'' = u^2 (e1r (x1^2 + 5 x1 + 17 + 36 q1) - e2r (x2^2 + 5 x2 + 17 + 36 q2))
// (|x2| >= 1; below, A'' = u^2 e2r (x2^2 + 2 x2 + 2) - (I/r)'' and B'' = 3 (I/r)'' + u^2 (e1r
// (x1^2 + 2 x1 + 2) - e2r (x2^2 + 2 x2 + 2)), the branch of the forward kernel); the speed
// derivatives of A, B (those of the single layer) differentiated in R:
//   dA'/dc1 = u (x1 + 1) e1r / c1, dA'/dc2 = u (1 + x2 - x2^2) e2r / c2,
//   dB'/dc1 = -u (x1^2 + x1 + 1) e1r / c1, dB'/dc2 = u (x2^2 + x2 + 1) e2r / c2.
// With lamc = c1^2 - 2 c2^2, G = A' + B' + 2 B u: P1 = lamc G + 2 c2^2 B u, P2 = c2^2 (A' + B u),
// P3 = 2 c2^2 (B' - 2 B u), differentiated term by term (lamc and c2^2 depend on the speeds).
struct TDer {
    zd P[3], Pr[3], Pc1[3], Pc2[3];
};

__device__ __forceinline__ void traction_der(double R, double Rinv, zd s, zd sinv, const Mat<double>& M, TDer& o)
{
    zd A, B, Ad, Bd;
    kernel_AB<double, true>(R, Rinv, s, sinv, M, A, B, Ad, Bd);
    const zd x1 = s * (R * M.ic1), x2 = s * (R * M.ic2);
    const zd e1r = M_<double>::cexpm(x1) * (M.ic1s * Rinv), e2r = M_<double>::cexpm(x2) * (M.ic2s * Rinv);
    const double u = Rinv, u2 = Rinv * Rinv;
    const zd one = {1.0, 0.0};
    zd Add, Bdd;
    if (abs2(x2) < 1.0) {
        zd p1, p2;
        psi2(x1, x2, p1, p2);
        const zd Irr = (p2 * M.ic2s - p1 * M.ic1s) * (u2 * u);
        const zd f1 = x1 * x1 + 2.0 * x1 + zd{2.0, 0.0}, f2 = x2 * x2 + 2.0 * x2 + zd{2.0, 0.0};
        Add = (e2r * f2) * u2 - Irr;
        Bdd = 3.0 * Irr + (e1r * f1 - e2r * f2) * u2;
    } else {
        const zd y1 = sinv * (M.c1 * Rinv), y2 = sinv * (M.c2 * Rinv);
        const zd q1 = y1 + y1 * y1, q2 = y2 + y2 * y2;
        Add = (e2r * (x2 * x2 + 3.0 * x2 + 12.0 * q2 + zd{7.0, 0.0}) - e1r * (x1 + 12.0 * q1 + zd{5.0, 0.0})) * u2;
        Bdd = (e1r * (x1 * x1 + 5.0 * x1 + 36.0 * q1 + zd{17.0, 0.0}) -
               e2r * (x2 * x2 + 5.0 * x2 + 36.0 * q2 + zd{17.0, 0.0})) * u2;
    }
    const zd A1 = e1r * (-M.ic1), A2 = (e2r * (x2 - one)) * M.ic2;
    const zd B1 = (e1r * (x1 + one)) * M.ic1, B2 = (e2r * (x2 + one)) * (-M.ic2);
    const zd A1d = (e1r * (x1 + one)) * (u * M.ic1), A2d = (e2r * (one + x2 - x2 * x2)) * (u * M.ic2);
    const zd B1d = (e1r * (x1 * x1 + x1 + one)) * (-u * M.ic1), B2d = (e2r * (x2 * x2 + x2 + one)) * (u * M.ic2);
    const double lamc = M.lamc, c2s = M.c2s, c1 = M.c1, c2 = M.c2;
    const zd Bu = B * u, G = Ad + Bd + 2.0 * Bu;
    o.P[0] = lamc * G + (2.0 * c2s) * Bu;
    o.P[1] = c2s * (Ad + Bu);
    o.P[2] = (2.0 * c2s) * (Bd - 2.0 * Bu);
    o.Pr[0] = lamc * (Add + Bdd + (2.0 * u) * (Bd - Bu)) + (2.0 * c2s * u) * (Bd - Bu);
    o.Pr[1] = c2s * (Add + u * (Bd - Bu));
    o.Pr[2] = (2.0 * c2s) * (Bdd - (2.0 * u) * (Bd - Bu));
    o.Pc1[0] = (2.0 * c1) * G + lamc * (A1d + B1d + (2.0 * u) * B1) + (2.0 * c2s * u) * B1;
    o.Pc1[1] = c2s * (A1d + u * B1);
    o.Pc1[2] = (2.0 * c2s) * (B1d - (2.0 * u) * B1);
    o.Pc2[0] = (-4.0 * c2) * G + lamc * (A2d + B2d + (2.0 * u) * B2) + (4.0 * c2) * Bu + (2.0 * c2s * u) * B2;
    o.Pc2[1] = (2.0 * c2) * (Ad + Bu) + c2s * (A2d + u * B2);
    o.Pc2[2] = (4.0 * c2) * (Bd - 2.0 * Bu) + (2.0 * c2s) * (B2d - (2.0 * u) * B2);
}

// Regular and near pairs of the double layer (i != j; pair classes held fixed), the layout of
// k_adjoint_v.  With W = w_i x_j^T (one right-hand side), rh = r / R, dr/dn = rh.n and
// 4 pi v = P1 S1 + P2 S2 + P3 S3, S1 = rh^T W n, S2 = tr(W) dr/dn + n^T W rh, S3 = rh^T W rh dr/dn:
//   4 pi grad_r v = rh (P1' S1 + P2' S2 + P3' S3) + (cw w_i + cx x_j + cn n - (P1 S1 + P2 S2 +
//                   3 P3 S3) rh) / R,
//   cw = P1 (x.n) + P3 dr/dn (x.rh), cx = P2 (w.n) + P3 dr/dn (w.rh), cn = P2 (w.x) + P3 (w.rh)(x.rh);
//   4 pi grad_n v = P1 (w.rh) x_j + P2 (x.rh) w_i + cn rh,
// and the normal n_j = N / |N|, N = (P_1 - P_0) x (P_2 - P_0), moves with vertex a as
// dn = (I - n n^T)(dP_a x (P_{a+1} - P_{a+2})) / |N|.  Outputs as k_adjoint_v.
__global__ __launch_bounds__(WG, 2) void k_adjoint_k(DevCtx c, int nrhs, const zd* __restrict__ w,
                                                  const zd* __restrict__ x, double* __restrict__ gJ,
                                                  double* __restrict__ gI, double* __restrict__ gM)
{
    __shared__ double red[WG / 64][9];
    const Geo& g = c.geo;
    const int K = g.K, L = c.fr.L;
    const size_t M = 3 * (size_t)K;
    const int i = blockIdx.x * WG + threadIdx.x;
    const bool act = i < K;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int j0 = blockIdx.y * JB, j1 = min(K, j0 + JB);
    const double pref = c.md.inv4pi;
    double ci[3] = {0.0, 0.0, 0.0}, mat[4] = {0.0, 0.0, 0.0, 0.0};
    const double xi[3] = {act ? g.cx[i] : 0.0, act ? g.cy[i] : 0.0, act ? g.cz[i] : 0.0};
    for (int j = j0; j < j1; ++j) {
        double gj[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) gj[t] = 0.0;
        if (act && i != j) {
            double P[3][3];
            for (int a = 0; a < 3; ++a) {
                P[a][0] = g.vx[a * K + j];
                P[a][1] = g.vy[a * K + j];
                P[a][2] = g.vz[a * K + j];
            }
            const double n[3] = {g.nx[j], g.ny[j], g.nz[j]};
            const double e1[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
            const double e2[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
            double dA[3][3];
            dA[1][0] = 0.5 * (e2[1] * n[2] - e2[2] * n[1]);
            dA[1][1] = 0.5 * (e2[2] * n[0] - e2[0] * n[2]);
            dA[1][2] = 0.5 * (e2[0] * n[1] - e2[1] * n[0]);
            dA[2][0] = 0.5 * (n[1] * e1[2] - n[2] * e1[1]);
            dA[2][1] = 0.5 * (n[2] * e1[0] - n[0] * e1[2]);
            dA[2][2] = 0.5 * (n[0] * e1[1] - n[1] * e1[0]);
            for (int k = 0; k < 3; ++k) dA[0][k] = -(dA[1][k] + dA[2][k]);
            const int m = pair_class(g, i, j, c.qt);
            const int nsub = 1 << (2 * m);
            const double wsub = g.area[j] * pref / (double)nsub;
            double gn[3] = {0.0, 0.0, 0.0};  // d Re S / d n_j of this pair
#pragma unroll 1
            for (int u = 0; u < nsub; ++u) {
            double Sb[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
#pragma unroll 1
            for (int lev = m - 1; lev >= 0; --lev) {
                const int ch = (u >> (2 * lev)) & 3;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double p0 = Sb[0][a], p1 = Sb[1][a], p2 = Sb[2][a];
                    const double m01 = 0.5 * (p0 + p1), m12 = 0.5 * (p1 + p2), m20 = 0.5 * (p2 + p0);
                    if (ch == 0) { Sb[1][a] = m01; Sb[2][a] = m20; }
                    else if (ch == 1) { Sb[0][a] = m01; Sb[2][a] = m12; }
                    else if (ch == 2) { Sb[0][a] = m20; Sb[1][a] = m12; }
                    else { Sb[0][a] = m01; Sb[1][a] = m12; Sb[2][a] = m20; }
                }
            }
#pragma unroll 1
            for (int q = 0; q < 7; ++q) {
                const double* bq = c.qt.b7 + 3 * q;
                double b[3], y[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) b[a] = bq[0] * Sb[0][a] + bq[1] * Sb[1][a] + bq[2] * Sb[2][a];
#pragma unroll
                for (int k = 0; k < 3; ++k) y[k] = b[0] * P[0][k] + b[1] * P[1][k] + b[2] * P[2][k];
                const double r[3] = {y[0] - xi[0], y[1] - xi[1], y[2] - xi[2]};
                const double R2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                const double Rinv = 1.0 / sqrt(R2), R = R2 * Rinv;
                const double rh[3] = {r[0] * Rinv, r[1] * Rinv, r[2] * Rinv};
                const double rn = rh[0] * n[0] + rh[1] * n[1] + rh[2] * n[2];
                double Gr[3] = {0.0, 0.0, 0.0}, Gn[3] = {0.0, 0.0, 0.0}, V = 0.0, Vi = 0.0, m1 = 0.0, m2 = 0.0;
#pragma unroll 1
                for (int l = 0; l < L; ++l) {
                    TDer T;
                    traction_der(R, Rinv, c.fr.s[l], c.fr.sinv[l], c.md, T);
#pragma unroll 1
                    for (int rr = 0; rr < nrhs; ++rr) {
                        const zd* up = w + ((size_t)rr * L + l) * M + 3 * (size_t)i;
                        const zd* vp = x + ((size_t)rr * L + l) * M + 3 * (size_t)j;
                        const zd uu[3] = {up[0], up[1], up[2]}, vv[3] = {vp[0], vp[1], vp[2]};
                        const zd wn = uu[0] * n[0] + uu[1] * n[1] + uu[2] * n[2];
                        const zd xn = vv[0] * n[0] + vv[1] * n[1] + vv[2] * n[2];
                        const zd wh = uu[0] * rh[0] + uu[1] * rh[1] + uu[2] * rh[2];
                        const zd xh = vv[0] * rh[0] + vv[1] * rh[1] + vv[2] * rh[2];
                        const zd be = uu[0] * vv[0] + uu[1] * vv[1] + uu[2] * vv[2];
                        const zd de = wh * xh;
                        const zd S1 = wh * xn, S2 = be * rn + wn * xh, S3 = de * rn;
                        const zd val = T.P[0] * S1 + T.P[1] * S2 + T.P[2] * S3;
                        const zd rad = T.Pr[0] * S1 + T.Pr[1] * S2 + T.Pr[2] * S3;
                        const zd cw = T.P[0] * xn + T.P[2] * (rn * xh);
                        const zd cxj = T.P[1] * wn + T.P[2] * (rn * wh);
                        const zd cn = T.P[1] * be + T.P[2] * de;
                        const zd ch = -(T.P[0] * S1 + T.P[1] * S2 + 3.0 * (T.P[2] * S3));
                        const zd a1 = T.P[0] * wh, a2 = T.P[1] * xh;
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            Gr[k] += rh[k] * rad.re + Rinv * (cw * uu[k] + cxj * vv[k] + ch * rh[k]).re + Rinv * n[k] * cn.re;
                            Gn[k] += (a1 * vv[k] + a2 * uu[k]).re + rh[k] * cn.re;
                        }
                        V += val.re;
                        Vi += val.im;
                        m1 += (T.Pc1[0] * S1 + T.Pc1[1] * S2 + T.Pc1[2] * S3).re;
                        m2 += (T.Pc2[0] * S1 + T.Pc2[1] * S2 + T.Pc2[2] * S3).re;
                    }
                }
                const double w7 = c.qt.w7[q] * pref / (double)nsub, wA = c.qt.w7[q] * wsub;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double gk = wA * Gr[k];
                    ci[k] -= gk;
                    gn[k] += wA * Gn[k];
#pragma unroll
                    for (int a = 0; a < 3; ++a) gj[3 * a + k] += b[a] * gk + w7 * V * dA[a][k];
                }
                mat[0] += wA * m1;
                mat[1] += wA * m2;
                mat[2] += wA * V;
                mat[3] += wA * Vi;
            }
            }
            // the normal's motion with the vertices
            const double iN = 0.5 / g.area[j];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
                const double d[3] = {P[a1][0] - P[a2][0], P[a1][1] - P[a2][1], P[a1][2] - P[a2][2]};
                // (e_k x d) . gn - (n . (e_k x d)) (n . gn) = e_k . (d x gn - (n.gn) (d x n))
                const double ng = n[0] * gn[0] + n[1] * gn[1] + n[2] * gn[2];
                const double dg[3] = {d[1] * gn[2] - d[2] * gn[1], d[2] * gn[0] - d[0] * gn[2], d[0] * gn[1] - d[1] * gn[0]};
                const double dn[3] = {d[1] * n[2] - d[2] * n[1], d[2] * n[0] - d[0] * n[2], d[0] * n[1] - d[1] * n[0]};
#pragma unroll
                for (int k = 0; k < 3; ++k) gj[3 * a + k] += iN * (dg[k] - ng * dn[k]);
            }
        }
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const double sv = wsum(gj[t]);
            if (lane == 0) red[wv][t] = sv;
        }
        __syncthreads();
        if (threadIdx.x < 9) {
            double sv = 0.0;
            for (int q = 0; q < WG / 64; ++q) sv += red[q][threadIdx.x];
            gJ[((size_t)blockIdx.x * K + j) * 9 + threadIdx.x] = sv;
        }
        __syncthreads();
    }
    if (act)
        for (int k = 0; k < 3; ++k) gI[((size_t)blockIdx.y * K + i) * 3 + k] = ci[k];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const double sv = wsum(mat[t]);
        if (lane == 0) red[wv][t] = sv;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double sv = 0.0;
        for (int q = 0; q < WG / 64; ++q) sv += red[q][threadIdx.x];
        gM[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 4 + threadIdx.x] = sv;
    }
}

// Contraction of 4 pi T(r, n) with a general 3 x 3 W (sum over the right-hand sides of
// w x^T) and its derivatives: with rh, dr/dn = rh.n, alpha = rh^T W n, beta = tr W, gamma =
// n^T W rh, delta = rh^T W rh, S = (alpha, beta dr/dn + gamma, delta dr/dn),
//   val = P.S, grad_r = rh (P'.S) + (P1 (W n - rh alpha) + P2 (beta (n - rh dr/dn) + W^T n -
//   rh gamma) + P3 (dr/dn ((W + W^T) rh - 2 rh delta) + delta (n - rh dr/dn))) / R,
//   grad_n = P1 W^T rh + P2 (beta rh + W rh) + P3 delta rh,   d/dc = (dP/dc).S.
struct TCon {
    zd val, c1, c2;
    double gr[3], gn[3];  // real parts
};

__device__ __forceinline__ void tcontract(const zd W[9], const double rh[3], const double n[3], double Rinv,
                                          const zd P[3], const zd Pr[3], const zd Pc1[3], const zd Pc2[3], TCon& o)
{
    zd Wn[3], WTn[3], Wh[3], WTh[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        Wn[a] = W[3 * a] * n[0] + W[3 * a + 1] * n[1] + W[3 * a + 2] * n[2];
        Wh[a] = W[3 * a] * rh[0] + W[3 * a + 1] * rh[1] + W[3 * a + 2] * rh[2];
        WTn[a] = W[a] * n[0] + W[3 + a] * n[1] + W[6 + a] * n[2];
        WTh[a] = W[a] * rh[0] + W[3 + a] * rh[1] + W[6 + a] * rh[2];
    }
    const double rn = rh[0] * n[0] + rh[1] * n[1] + rh[2] * n[2];
    const zd al = rh[0] * Wn[0] + rh[1] * Wn[1] + rh[2] * Wn[2];
    const zd be = W[0] + W[4] + W[8];
    const zd ga = n[0] * Wh[0] + n[1] * Wh[1] + n[2] * Wh[2];
    const zd de = rh[0] * Wh[0] + rh[1] * Wh[1] + rh[2] * Wh[2];
    const zd S1 = al, S2 = be * rn + ga, S3 = de * rn;
    o.val = P[0] * S1 + P[1] * S2 + P[2] * S3;
    o.c1 = Pc1[0] * S1 + Pc1[1] * S2 + Pc1[2] * S3;
    o.c2 = Pc2[0] * S1 + Pc2[1] * S2 + Pc2[2] * S3;
    const zd rad = Pr[0] * S1 + Pr[1] * S2 + Pr[2] * S3;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const zd t = P[0] * (Wn[k] - rh[k] * al) + P[1] * (be * (n[k] - rh[k] * rn) + WTn[k] - rh[k] * ga) +
                     P[2] * (rn * (Wh[k] + WTh[k] - (2.0 * rh[k]) * de) + de * (n[k] - rh[k] * rn));
        o.gr[k] = rh[k] * rad.re + Rinv * t.re;
        o.gn[k] = (P[0] * WTh[k] + P[1] * (be * rh[k] + Wh[k]) + P[2] * (de * rh[k])).re;
    }
}

// Self pairs of the double layer, the derivative of the principal-value integral: the element
// stays flat under a perturbation of its vertices; with the collocation point x (centroid) and
// y = sum_a lambda_a(y) P_a,
//   dE/dP_a = PV int grad_r T(y - x, n) (lambda_a(y) - 1/3) dy + PV int grad_n T dy . dn/dP_a
//             + (dA/dP_a / A) E,   dE/dc = PV int dT/dc dy.
// Each integrand is G(theta) / rho^2 + O(1) at x with G odd in the direction (T = T_0 / R^2 +
// O(1): A' and B / R have no 1/R term), so the polar rule of the forward self entry takes it,
// per angular line w_theta [sum_rho w_rho rho F + G (ln R - crho)], with G from the static
// coefficients P_0 = (c2^2/c1^2, -c2^2/c1^2, -3 (1 - c2^2/c1^2)), P'_0 = -2 P_0 at unit
// distance.  Thread per element j, frequencies outermost (W_l = sum_r w x^T of the element);
// out[j][13] as k_adjoint_self, with the free term I/2 in the value when free_term.
__global__ __launch_bounds__(64) void k_adjoint_kself(DevCtx c, int free_term, int nrhs, const zd* __restrict__ w,
                                                      const zd* __restrict__ x, double* __restrict__ out)
{
    const Geo& g = c.geo;
    const QuadTab& Q = c.qt;
    const Mat<double>& Md = c.md;
    const int K = g.K, L = c.fr.L;
    const size_t Mv = 3 * (size_t)K;
    const int j = blockIdx.x * 64 + threadIdx.x;
    if (j >= K) return;
    const double pref = Md.inv4pi;
    double P[3][3];
    for (int a = 0; a < 3; ++a) {
        P[a][0] = g.vx[a * K + j];
        P[a][1] = g.vy[a * K + j];
        P[a][2] = g.vz[a * K + j];
    }
    const double xc[3] = {g.cx[j], g.cy[j], g.cz[j]};
    const double n[3] = {g.nx[j], g.ny[j], g.nz[j]};
    // static coefficients and their speed derivatives
    const double gam = Md.c2s * Md.ic1s;
    const double dg1 = -2.0 * gam * Md.ic1, dg2 = 2.0 * Md.c2 * Md.ic1s;
    const zd p0[3] = {{gam, 0.0}, {-gam, 0.0}, {-3.0 * (1.0 - gam), 0.0}};
    const zd p0r[3] = {{-2.0 * gam, 0.0}, {2.0 * gam, 0.0}, {6.0 * (1.0 - gam), 0.0}};
    const zd p0c1[3] = {{dg1, 0.0}, {-dg1, 0.0}, {3.0 * dg1, 0.0}};
    const zd p0c2[3] = {{dg2, 0.0}, {-dg2, 0.0}, {3.0 * dg2, 0.0}};
    double gP[9], gN[3] = {0.0, 0.0, 0.0}, V = 0.0, Vi = 0.0, m1 = 0.0, m2 = 0.0;
    zd trW = {0.0, 0.0};  // sum_{r, l} w . x of the element (the free term's share)
    for (int t = 0; t < 9; ++t) gP[t] = 0.0;
#pragma unroll 1
    for (int l = 0; l < L; ++l) {
        zd W[9];
        for (int t = 0; t < 9; ++t) W[t] = {0.0, 0.0};
        for (int rr = 0; rr < nrhs; ++rr) {
            const zd* up = w + ((size_t)rr * L + l) * Mv + 3 * (size_t)j;
            const zd* vp = x + ((size_t)rr * L + l) * Mv + 3 * (size_t)j;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) W[3 * a + b] = fma_c(up[a], vp[b], W[3 * a + b]);
        }
        const zd sl = c.fr.s[l], sinvl = c.fr.sinv[l];
#pragma unroll 1
        for (int sa = 0; sa < 3; ++sa) {
            const int sb = (sa + 1) % 3;
            double t[3] = {P[sb][0] - P[sa][0], P[sb][1] - P[sa][1], P[sb][2] - P[sa][2]};
            const double le = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
            for (int k = 0; k < 3; ++k) t[k] /= le;
            const double proj = (xc[0] - P[sa][0]) * t[0] + (xc[1] - P[sa][1]) * t[1] + (xc[2] - P[sa][2]) * t[2];
            double foot[3], p[3];
            for (int k = 0; k < 3; ++k) {
                foot[k] = P[sa][k] + proj * t[k];
                p[k] = foot[k] - xc[k];
            }
            const double d = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
            for (int k = 0; k < 3; ++k) p[k] /= d;
            const double qa = (P[sa][0] - foot[0]) * t[0] + (P[sa][1] - foot[1]) * t[1] + (P[sa][2] - foot[2]) * t[2];
            const double qb = (P[sb][0] - foot[0]) * t[0] + (P[sb][1] - foot[1]) * t[1] + (P[sb][2] - foot[2]) * t[2];
            const double ta = atan2(qa, d), tb = atan2(qb, d);
            const double hth = 0.5 * (tb - ta), mth = 0.5 * (ta + tb);
#pragma unroll 1
            for (int it = 0; it < Q.nt; ++it) {
                const double th = mth + hth * Q.tx[it];
                const double wth = hth * Q.tw[it];
                double sn, cs;
                sincos(th, &sn, &cs);
                const double Rl = d / cs;
                const double rh[3] = {cs * p[0] + sn * t[0], cs * p[1] + sn * t[1], cs * p[2] + sn * t[2]};
                double lam1[3];  // lambda_b - 1/3 per unit distance along rh
                {
                    const double y1[3] = {xc[0] + rh[0], xc[1] + rh[1], xc[2] + rh[2]};
                    for (int b = 0; b < 3; ++b) lam1[b] = bary_at(g, j, b, y1) - 1.0 / 3.0;
                }
                // leading parts: w_theta G (ln R - crho)
                {
                    TCon o;
                    tcontract(W, rh, n, 1.0, p0, p0r, p0c1, p0c2, o);
                    const double cw = wth * (log(Rl) - Q.crho) * pref;
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        gN[k] += cw * o.gn[k];
#pragma unroll
                        for (int b = 0; b < 3; ++b) gP[3 * b + k] += cw * o.gr[k] * lam1[b];
                    }
                    V += cw * o.val.re;
                    Vi += cw * o.val.im;
                    m1 += cw * o.c1.re;
                    m2 += cw * o.c2.re;
                }
#pragma unroll 1
                for (int ir = 0; ir < Q.nr; ++ir) {
                    const double rho = 0.5 * Rl * (1.0 + Q.rx[ir]);
                    const double wq = wth * (0.5 * Rl * Q.rw[ir]) * rho * pref;
                    TDer T;
                    traction_der(rho, 1.0 / rho, sl, sinvl, Md, T);
                    TCon o;
                    tcontract(W, rh, n, 1.0 / rho, T.P, T.Pr, T.Pc1, T.Pc2, o);
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        gN[k] += wq * o.gn[k];
#pragma unroll
                        for (int b = 0; b < 3; ++b) gP[3 * b + k] += wq * o.gr[k] * (rho * lam1[b]);
                    }
                    V += wq * o.val.re;
                    Vi += wq * o.val.im;
                    m1 += wq * o.c1.re;
                    m2 += wq * o.c2.re;
                }
            }
        }
        trW += W[0] + W[4] + W[8];
    }
    // area term (of the integral, without the free term) and the normal's motion
    const double e1[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
    const double e2[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
    double dA[3][3];
    dA[1][0] = 0.5 * (e2[1] * n[2] - e2[2] * n[1]);
    dA[1][1] = 0.5 * (e2[2] * n[0] - e2[0] * n[2]);
    dA[1][2] = 0.5 * (e2[0] * n[1] - e2[1] * n[0]);
    dA[2][0] = 0.5 * (n[1] * e1[2] - n[2] * e1[1]);
    dA[2][1] = 0.5 * (n[2] * e1[0] - n[0] * e1[2]);
    dA[2][2] = 0.5 * (n[0] * e1[1] - n[1] * e1[0]);
    for (int k = 0; k < 3; ++k) dA[0][k] = -(dA[1][k] + dA[2][k]);
    const double ia = 1.0 / g.area[j], iN = 0.5 * ia;
    const double ng = n[0] * gN[0] + n[1] * gN[1] + n[2] * gN[2];
    double* o = out + (size_t)j * 13;
    for (int a = 0; a < 3; ++a) {
        const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
        const double dd[3] = {P[a1][0] - P[a2][0], P[a1][1] - P[a2][1], P[a1][2] - P[a2][2]};
        const double dg[3] = {dd[1] * gN[2] - dd[2] * gN[1], dd[2] * gN[0] - dd[0] * gN[2], dd[0] * gN[1] - dd[1] * gN[0]};
        const double dn[3] = {dd[1] * n[2] - dd[2] * n[1], dd[2] * n[0] - dd[0] * n[2], dd[0] * n[1] - dd[1] * n[0]};
        for (int k = 0; k < 3; ++k) o[3 * a + k] = gP[3 * a + k] + V * dA[a][k] * ia + iN * (dg[k] - ng * dn[k]);
    }
    o[9] = m1;
    o[10] = m2;
    o[11] = V + (free_term ? 0.5 * trW.re : 0.0);
    o[12] = Vi + (free_term ? 0.5 * trW.im : 0.0);
}

// out[e][t] = sum over tiles of part[tile][e][t] (fixed order)
__global__ __launch_bounds__(WG) void k_sum_tiles(const double* __restrict__ part, int ntile, size_t n,
                                                  double* __restrict__ out)
{
    const size_t q = (size_t)blockIdx.x * WG + threadIdx.x;
    if (q >= n) return;
    double s = 0.0;
    for (int t = 0; t < ntile; ++t) s += part[(size_t)t * n + q];
    out[q] = s;
}

}  // namespace

void launch_mf_apply(const DevCtx& c, int op, bool transpose, int nrhs, const zd* x, zd* y, hipStream_t st)
{
    const dim3 grid((unsigned)((c.geo.K + WG - 1) / WG), (unsigned)c.fr.L);
    if (transpose) hipLaunchKernelGGL(k_mf_apply<true>, grid, dim3(WG), 0, st, c, op, nrhs, x, y);
    else hipLaunchKernelGGL(k_mf_apply<false>, grid, dim3(WG), 0, st, c, op, nrhs, x, y);
    BEM_HIP_TRY(hipGetLastError());
}

void launch_mf_apply_kl(const DevCtx& c, const int* tri, int nnodes, int nrhs, const zd* g, zd* y, bool free_term,
                        hipStream_t st)
{
    const int K = c.geo.K;
    if (K <= 0 || nrhs <= 0) return;
    hipLaunchKernelGGL(k_mf_apply_kl, dim3((K + WG - 1) / WG, c.fr.L), dim3(WG), 0, st, c, tri, nnodes, nrhs, g, y,
                       free_term ? 1 : 0);
    BEM_HIP_TRY(hipGetLastError());
}

size_t adjoint_work_doubles(int K)
{
    const size_t ti = (K + WG - 1) / WG, tj = (K + JB - 1) / JB;
    return ti * K * 9 + tj * K * 3 + ti * tj * 4 + (size_t)K * 13 + (size_t)K * 12;
}

// work: adjoint_work_doubles(K); on return (on the stream) sums[0 .. 12 K): per element 9
// vertex derivatives of the regular pairs as column element, then 3 centroid derivatives as
// row element; tiles[..]: the per-workgroup dc1, dc2, Re S, Im S (ntiles_out of them); self
// results [K][13].
void launch_adjoint_v(const DevCtx& c, int nrhs, const zd* w, const zd* x, double* work, double** sums, double** tiles,
                      int* ntiles_out, double** self_out,
                      hipStream_t st)
{
    const int K = c.geo.K;
    const unsigned ti = (unsigned)((K + WG - 1) / WG), tj = (unsigned)((K + JB - 1) / JB);
    double* gJ = work;
    double* gI = gJ + (size_t)ti * K * 9;
    double* gM = gI + (size_t)tj * K * 3;
    double* so = gM + (size_t)ti * tj * 4;
    double* sum = so + (size_t)K * 13;
    hipLaunchKernelGGL(k_adjoint_v, dim3(ti, tj), dim3(WG), 0, st, c, nrhs, w, x, gJ, gI, gM);
    BEM_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_adjoint_self, dim3((unsigned)(((size_t)K + 63) / 64)), dim3(64), 0, st, c, nrhs, w, x, so);
    BEM_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_sum_tiles, dim3((unsigned)((9 * (size_t)K + WG - 1) / WG)), dim3(WG), 0, st, gJ, (int)ti,
                       9 * (size_t)K, sum);
    BEM_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_sum_tiles, dim3((unsigned)((3 * (size_t)K + WG - 1) / WG)), dim3(WG), 0, st, gI, (int)tj,
                       3 * (size_t)K, sum + 9 * (size_t)K);
    BEM_HIP_TRY(hipGetLastError());
    *sums = sum;
    *tiles = gM;
    *ntiles_out = (int)(ti * tj);
    *self_out = so;
}

// The double layer's adjoint (op K, or I/2 + K with free_term), same work layout and outputs
// as launch_adjoint_v.
void launch_adjoint_k(const DevCtx& c, bool free_term, int nrhs, const zd* w, const zd* x, double* work, double** sums,
                      double** tiles, int* ntiles_out, double** self_out, hipStream_t st)
{
    const int K = c.geo.K;
    const unsigned ti = (unsigned)((K + WG - 1) / WG), tj = (unsigned)((K + JB - 1) / JB);
    double* gJ = work;
    double* gI = gJ + (size_t)ti * K * 9;
    double* gM = gI + (size_t)tj * K * 3;
    double* so = gM + (size_t)ti * tj * 4;
    double* sum = so + (size_t)K * 13;
    hipLaunchKernelGGL(k_adjoint_k, dim3(ti, tj), dim3(WG), 0, st, c, nrhs, w, x, gJ, gI, gM);
    BEM_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_adjoint_kself, dim3((unsigned)(((size_t)K + 63) / 64)), dim3(64), 0, st, c, free_term ? 1 : 0,
                       nrhs, w, x, so);
    BEM_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_sum_tiles, dim3((unsigned)((9 * (size_t)K + WG - 1) / WG)), dim3(WG), 0, st, gJ, (int)ti,
                       9 * (size_t)K, sum);
    BEM_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_sum_tiles, dim3((unsigned)((3 * (size_t)K + WG - 1) / WG)), dim3(WG), 0, st, gI, (int)tj,
                       3 * (size_t)K, sum + 9 * (size_t)K);
    BEM_HIP_TRY(hipGetLastError());
    *sums = sum;
    *tiles = gM;
    *ntiles_out = (int)(ti * tj);
    *self_out = so;
}

}  // namespace bem
