// recomp.hip -- recompression of the per-slice ACA factors of a face (Sec. 3: the cross
// approximation U V^H of a face is recompressed by QR factorisations and an SVD of the
// small core, eq. (ACA)).  One workgroup of 1024 threads per face; the kc x kc core
// (kc <= 96 ACA columns) lives in LDS, U and V in the face's scratch slot.
//
//   U D_U^-1 = Q_U T_U, V D_V^-1 = Q_V T_V   CholeskyQR of the column-scaled ACA columns,
//                                            repeated once (CholeskyQR2) when a Cholesky
//                                            pivot of the unit-diagonal Gram is below 1e-10
//   M = R_U R_V^H, R = T D                   the core
//   M P = Q_M R                              Householder QR with column pivoting, stopped once
//                                            the remaining columns have norm <= tol / 4:
//                                            M ~ Q_M B, B = R_top P^T (k' rows)
//   B^H VJ = W                               one-sided Jacobi on the k' columns of B^H
//                                            (W_s orthogonal, |W_s| = sigma_s, VJ unitary)
//   M ~ sum_s (Q_M VJ_s) sigma_s (W_s / sigma_s)^H with VJ_s = B W_s / sigma_s^2,
//   truncated at tol with the dropped QR part counted in the tail, so that
//   Ubar_s = Q_U Q_M VJ_s sigma_s and Vbar_s = Q_V W_s / sigma_s.
// The factors overwrite the face (row-major, the face's precision) when they take less
// memory than the dense face.
//
// Each step of the column-sequential parts (Cholesky, pivoted QR, Jacobi rounds,
// back-substitution, reflector application) ends in one workgroup barrier; the serial part
// of a pivoted-QR step (pivot, reflector) runs in wavefront 0 alone.
#include "aca3d.hpp"

namespace bem {

namespace {

constexpr int NT = 1024;        // threads of a recompression workgroup
constexpr int NW = NT / 64;     // its wavefronts
constexpr int KF = 96;          // largest core (ACA columns)

// The pivoted QR of the core stops once its remaining columns are below QRCP_FRAC tol; the
// SVD truncation of the kept rows then has sqrt(1 - QRCP_FRAC^2) of the tolerance left.
constexpr double QRCP_FRAC = 0.25;

// Smallest Cholesky pivot of the column-scaled Gram (unit diagonal) that a single CholeskyQR
// accepts: below it (condition above ~1e5) the factor is refined by a second pass.
constexpr double CQ2_PIVOT = 1e-10;

template <typename T> __device__ __forceinline__ zd ldz(const cx<T>* p) { return {(double)p->re, (double)p->im}; }
template <typename T> __device__ __forceinline__ void stz(cx<T>* p, zd v) { *p = {(T)v.re, (T)v.im}; }

__device__ __forceinline__ double wsum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// orders the LDS accesses of the lanes of one wavefront (no hardware wait is needed: a
// wavefront's LDS instructions complete in order)
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

struct Rs {
    zd m[KF * KF];  // kc x kc working matrix, column-major with ld kc; Gram staging area
    zd tau[KF];     // reflector coefficients of the pivoted QR
    double sv[KF];  // column scales, squared column norms, singular values
    int order[KF];  // singular values by decreasing size
    int perm[KF];   // column order of the pivoted QR
    double s;
    int piv, flag;
};

// Lm = X^H X (kc x kc, full Hermitian) for X (rows x kc, column-major, global).  A thread
// owns up to two 2 x 2 tiles of the upper triangle; X is staged through Lm in row chunks.
__device__ void gram(const zd* X, int rows, int kc, zd* Lm)
{
    const int nt = (kc + 1) >> 1, ntri = nt * (nt + 1) / 2, kp = 2 * nt;
    const int cr = min(rows, (KF * KF) / kp);
    int ti[2], tj[2];
    bool act[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int tt = threadIdx.x + h * NT;
        act[h] = tt < ntri;
        int j = 0;
        if (act[h]) {
            j = (int)((sqrt(8.0 * tt + 1.0) - 1.0) * 0.5);
            while ((j + 1) * (j + 2) / 2 <= tt) ++j;
            while (j * (j + 1) / 2 > tt) --j;
        }
        tj[h] = j;
        ti[h] = act[h] ? tt - j * (j + 1) / 2 : 0;
    }
    zd acc[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[h][u] = {0.0, 0.0};
    for (int r0 = 0; r0 < rows; r0 += cr) {
        const int nr = min(cr, rows - r0);
        __syncthreads();
        for (int q = threadIdx.x; q < nr * kp; q += NT) {
            const int c = q / nr, r = q - c * nr;
            Lm[r * kp + c] = c < kc ? X[(size_t)c * rows + r0 + r] : zd{0.0, 0.0};
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (!act[h]) continue;
            const zd* pa = Lm + 2 * ti[h];
            const zd* pb = Lm + 2 * tj[h];
            for (int r = 0; r < nr; ++r) {
                const zd a0 = pa[r * kp], a1 = pa[r * kp + 1], b0 = pb[r * kp], b1 = pb[r * kp + 1];
                acc[h][0] += conj_mul(a0, b0);
                acc[h][1] += conj_mul(a0, b1);
                acc[h][2] += conj_mul(a1, b0);
                acc[h][3] += conj_mul(a1, b1);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (!act[h]) continue;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = 2 * ti[h] + (u >> 1), j = 2 * tj[h] + (u & 1);
            if (i < kc && j < kc && i <= j) {
                Lm[(size_t)j * kc + i] = acc[h][u];
                Lm[(size_t)i * kc + j] = conj(acc[h][u]);
            }
        }
    }
    __syncthreads();
}

// Cholesky in place: Lm = R^H R with R upper (upper triangle, the strictly lower part
// zeroed); a pivot without positive mass gives a zero row.  Step k updates the trailing
// matrix from the unscaled row k (divided by the pivot) and scales row k - 1 with the pivot
// read one step earlier.  Returns the smallest pivot (before the square root).
__device__ double cholesky(zd* Lm, int kc)
{
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    double pmin = 1e300, pprev = 0.0;
    for (int k = 0; k < kc; ++k) {
        const double p = Lm[(size_t)k * kc + k].re;
        pmin = fmin(pmin, p);
        if (k > 0) {
            const int kr = k - 1;
            const double rk = pprev > 1e-24 ? sqrt(pprev) : 0.0;
            for (int j = kr + threadIdx.x; j < kc; j += NT) {
                zd* e = Lm + (size_t)j * kc + kr;
                *e = j == kr ? zd{rk, 0.0} : (rk > 0.0 ? *e * (1.0 / rk) : zd{0.0, 0.0});
            }
        }
        if (p > 1e-24) {
            const double ip = 1.0 / p;
            for (int j = k + 1 + ty; j < kc; j += 32) {
                const zd rj = Lm[(size_t)j * kc + k] * ip;
                for (int i = k + 1 + tx; i <= j; i += 32) Lm[(size_t)j * kc + i] -= conj_mul(Lm[(size_t)i * kc + k], rj);
            }
        }
        pprev = p;
        __syncthreads();
    }
    if (threadIdx.x == 0 && kc > 0) {
        zd* e = Lm + (size_t)(kc - 1) * kc + kc - 1;
        *e = {pprev > 1e-24 ? sqrt(pprev) : 0.0, 0.0};
    }
    for (int q = threadIdx.x; q < kc * kc; q += NT)
        if (q % kc > q / kc) Lm[q] = {0.0, 0.0};
    __syncthreads();
    return pmin;
}

// X (rows x kc, column-major, global) <- X R^{-1}, R upper in Lm; one row per thread, blocks
// of 8 columns; zero pivots give zero columns.
__device__ void trsm(zd* X, int rows, const zd* Lm, int kc)
{
    constexpr int NB = 8;
    for (int r = threadIdx.x; r < rows; r += NT) {
        for (int j0 = 0; j0 < kc; j0 += NB) {
            const int nb = min(NB, kc - j0);
            zd acc[NB];
#pragma unroll
            for (int t = 0; t < NB; ++t) acc[t] = t < nb ? X[(size_t)(j0 + t) * rows + r] : zd{0.0, 0.0};
            for (int i = 0; i < j0; ++i) {
                const zd x = X[(size_t)i * rows + r];
#pragma unroll
                for (int t = 0; t < NB; ++t)
                    if (t < nb) acc[t] -= x * Lm[(size_t)(j0 + t) * kc + i];
            }
#pragma unroll
            for (int t = 0; t < NB; ++t) {
                if (t >= nb) break;
#pragma unroll
                for (int u = 0; u < t; ++u) acc[t] -= acc[u] * Lm[(size_t)(j0 + t) * kc + j0 + u];
                const double d = Lm[(size_t)(j0 + t) * kc + j0 + t].re;
                acc[t] = d > 0.0 ? acc[t] * (1.0 / d) : zd{0.0, 0.0};
            }
#pragma unroll
            for (int t = 0; t < NB; ++t)
                if (t < nb) X[(size_t)(j0 + t) * rows + r] = acc[t];
        }
    }
    __syncthreads();
}

// Column scaling + CholeskyQR of X (rows x kc), repeated once when the first pass meets a
// pivot below CQ2_PIVOT.  On return Q = X T^{-1} with T upper in Tout (X holds X D^{-1}, or
// X D^{-1} R1^{-1} after two passes) and R = R_fact D in Rout, R_fact the triangular factor
// of X D^{-1}; both kc x kc column-major in global scratch.
__device__ void chol_qr(zd* X, int rows, int kc, zd* Rout, zd* Tout, Rs& L)
{
    zd* Lm = L.m;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int c = wv; c < kc; c += NW) {
        double s = 0.0;
        for (int r = lane; r < rows; r += 64) s += abs2(X[(size_t)c * rows + r]);
        s = wsum(s);
        if (lane == 0) L.sv[c] = sqrt(s);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < rows * kc; q += NT) {
        const double dc = L.sv[q / rows];
        X[q] = dc > 0.0 ? X[q] * (1.0 / dc) : zd{0.0, 0.0};
    }
    __syncthreads();
    gram(X, rows, kc, Lm);
    const double pmin = cholesky(Lm, kc);
    if (pmin >= CQ2_PIVOT) {
        for (int q = threadIdx.x; q < kc * kc; q += NT) {
            Tout[q] = Lm[q];
            Rout[q] = Lm[q] * L.sv[q / kc];
        }
        __syncthreads();
        return;
    }
    trsm(X, rows, Lm, kc);
    for (int q = threadIdx.x; q < kc * kc; q += NT) Tout[q] = Lm[q];  // R1 (for now)
    __syncthreads();
    gram(X, rows, kc, Lm);
    cholesky(Lm, kc);
    // Rout = R2 R1 D, then Tout = R2
    for (int q = threadIdx.x; q < kc * kc; q += NT) {
        const int i = q % kc, j = q / kc;
        zd s = {0.0, 0.0};
        for (int t = i; t <= j; ++t) s += Lm[(size_t)t * kc + i] * Tout[(size_t)j * kc + t];
        Rout[q] = i <= j ? s * L.sv[j] : zd{0.0, 0.0};
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kc * kc; q += NT) Tout[q] = Lm[q];
    __syncthreads();
}

// Householder QR with column pivoting of Lm (kc x kc, column-major) in place: reflectors
// H = I - tau v v^H with v[0] = 1 stored below the diagonal, stopped at the first step whose
// remaining columns have Frobenius norm <= delta.  Returns the number of steps; tau in L.tau,
// the column order in L.perm, the remaining squared norm in *rest2.
__device__ int qrcp(zd* Lm, int kc, double delta, Rs& L, double* rest2)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int c = wv; c < kc; c += NW) {
        double s = 0.0;
        for (int r = lane; r < kc; r += 64) s += abs2(Lm[(size_t)c * kc + r]);
        s = wsum(s);
        if (lane == 0) {
            L.sv[c] = s;
            L.perm[c] = c;
        }
    }
    __syncthreads();
    int j = 0;
    for (; j < kc; ++j) {
        if (wv == 0) {
            // remaining norm and pivot column
            double t = 0.0, best = -1.0;
            int p = 0x7fffffff;
            for (int c = j + lane; c < kc; c += 64) {
                const double v = L.sv[c];
                t += v;
                if (v > best || (v == best && c < p)) {
                    best = v;
                    p = c;
                }
            }
            t = wsum(t);
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                const double ob = __shfl_xor(best, o, 64);
                const int oi = __shfl_xor(p, o, 64);
                if (ob > best || (ob == best && oi < p)) {
                    best = ob;
                    p = oi;
                }
            }
            if (sqrt(fmax(t, 0.0)) <= delta) p = -1;
            if (p >= 0) {
                // reflector of the pivot column (rows j..): beta = -sign(Re alpha) ||x||
                zd* aj = Lm + (size_t)j * kc;
                zd* ap = Lm + (size_t)p * kc;
                double x2 = 0.0;
                for (int r = j + 1 + lane; r < kc; r += 64) x2 += abs2(ap[r]);
                x2 = wsum(x2);
                const zd al = ap[j];
                zd tau = {0.0, 0.0}, sc = {0.0, 0.0}, diag = al;
                if (x2 > 0.0 || al.im != 0.0) {
                    const double nrm = sqrt(abs2(al) + x2);
                    const double beta = al.re >= 0.0 ? -nrm : nrm;
                    tau = {(beta - al.re) / beta, -al.im / beta};
                    sc = zdiv(zd{1.0, 0.0}, al - zd{beta, 0.0});
                    diag = {beta, 0.0};
                }
                wave_sync();
                // swap columns j and p; column j takes beta and the reflector below it
                for (int r = lane; r < kc; r += 64) {
                    const zd vj = aj[r], vp = ap[r];
                    ap[r] = vj;
                    aj[r] = r < j ? vp : (r == j ? diag : vp * sc);
                }
                if (lane == 0) {
                    L.tau[j] = tau;
                    const double sv = L.sv[j];
                    L.sv[j] = L.sv[p];
                    L.sv[p] = sv;
                    const int pm = L.perm[j];
                    L.perm[j] = L.perm[p];
                    L.perm[p] = pm;
                }
            }
            if (lane == 0) L.piv = p;
        }
        __syncthreads();
        if (L.piv < 0) break;
        // apply H^H to the columns j + 1 .. kc - 1 (one wavefront per column), refresh norms
        const zd tc = conj(L.tau[j]);
        const zd* aj = Lm + (size_t)j * kc;
        for (int c = j + 1 + wv; c < kc; c += NW) {
            zd* ac = Lm + (size_t)c * kc;
            double wr = 0.0, wi = 0.0;
            for (int r = j + lane; r < kc; r += 64) {
                const zd v = r == j ? zd{1.0, 0.0} : aj[r];
                const zd t = conj_mul(v, ac[r]);
                wr += t.re;
                wi += t.im;
            }
            wr = wsum(wr);
            wi = wsum(wi);
            const zd f = tc * zd{wr, wi};
            double s = 0.0;
            for (int r = j + lane; r < kc; r += 64) {
                const zd v = r == j ? zd{1.0, 0.0} : aj[r];
                const zd a = ac[r] - v * f;
                ac[r] = a;
                if (r > j) s += abs2(a);
            }
            s = wsum(s);
            if (lane == 0) L.sv[c] = s;
        }
        __syncthreads();
    }
    double rs = 0.0;
    for (int c = j; c < kc; ++c) rs += L.sv[c];
    *rest2 = j < kc ? rs : 0.0;
    __syncthreads();
    return j;
}

// One-sided Jacobi on the ncol columns (length rows <= KF, stride ld) at Lm: Lm <- B VJ with
// orthogonal columns, rotations not accumulated.  A group of JG lanes per column pair (the
// pair's rows in registers), round-robin pair order, one barrier per round.
template <int JG>
__device__ void jacobi(zd* Lm, int rows, int ncol, int ld, Rs& L)
{
    constexpr int RPL = (KF + JG - 1) / JG;
    const int np = ncol + (ncol & 1);
    const int g = threadIdx.x / JG, gl = threadIdx.x % JG;
    if (ncol < 2) return;
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (threadIdx.x == 0) L.flag = 0;
        __syncthreads();
        for (int rnd = 0; rnd < np - 1; ++rnd) {
            for (int pr = g; pr < np / 2; pr += NT / JG) {
                int p, q;
                if (pr == 0) {
                    p = rnd;
                    q = np - 1;
                } else {
                    p = (rnd + pr) % (np - 1);
                    q = (rnd - pr + np - 1) % (np - 1);
                }
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                if (q >= ncol) continue;  // uniform within the lane group
                zd* mp = Lm + (size_t)p * ld;
                zd* mq = Lm + (size_t)q * ld;
                zd a[RPL], b[RPL];
                double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
#pragma unroll
                for (int t = 0; t < RPL; ++t) {
                    const int r = gl + JG * t;
                    a[t] = r < rows ? mp[r] : zd{0.0, 0.0};
                    b[t] = r < rows ? mq[r] : zd{0.0, 0.0};
                    al += abs2(a[t]);
                    be += abs2(b[t]);
                    const zd c = conj_mul(a[t], b[t]);
                    gr += c.re;
                    gi += c.im;
                }
#pragma unroll
                for (int o = 1; o < JG; o <<= 1) {
                    al += __shfl_xor(al, o, 64);
                    be += __shfl_xor(be, o, 64);
                    gr += __shfl_xor(gr, o, 64);
                    gi += __shfl_xor(gi, o, 64);
                }
                const double gabs = sqrt(gr * gr + gi * gi);
                if (!(gabs > 1e-12 * sqrt(al * be)) || gabs == 0.0) continue;
                if (gl == 0) L.flag = 1;
                const zd e = {gr / gabs, gi / gabs};
                const double zeta = (be - al) / (2.0 * gabs);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                const zd ce = conj(e);
#pragma unroll
                for (int u = 0; u < RPL; ++u) {
                    const int r = gl + JG * u;
                    if (r >= rows) break;
                    const zd bb = b[u] * ce;
                    mp[r] = c * a[u] - s * bb;
                    mq[r] = (s * a[u] + c * bb) * e;
                }
            }
            __syncthreads();
        }
        const int f = L.flag;
        __syncthreads();
        if (!f) break;
    }
}

// Y_h <- R_h^{-1} Y_h for up to two systems h (kk columns each, column s at Y_h + s kc, kc
// rows in LDS), R_h upper (kc x kc, column-major, global); right-looking from the last row,
// one barrier per row: step i subtracts column i of R times y_i / r_ii from the rows above,
// and the rows are divided by their pivots at the end (zero pivots: zero rows).
__device__ void backsub2(const zd* R0, zd* Y0, const zd* R1, zd* Y1, int kc, int kk)
{
    const int nsys = Y1 ? 2 : 1;
    for (int i = kc - 1; i >= 1; --i) {
        const int per = i * kk;
        for (int q = threadIdx.x; q < nsys * per; q += NT) {
            const bool h = q >= per;
            const int qq = h ? q - per : q;
            const int s = qq / i, t = qq - s * i;
            const zd* R = h ? R1 : R0;
            const double d = R[(size_t)i * kc + i].re;
            if (d > 0.0) {
                zd* y = (h ? Y1 : Y0) + (size_t)s * kc;
                y[t] -= R[(size_t)i * kc + t] * (y[i] * (1.0 / d));
            }
        }
        __syncthreads();
    }
    for (int q = threadIdx.x; q < nsys * kc * kk; q += NT) {
        const bool h = q >= kc * kk;
        const int qq = h ? q - kc * kk : q;
        const int i = qq % kc;
        const double d = (h ? R1 : R0)[(size_t)i * kc + i].re;
        zd* y = (h ? Y1 : Y0) + qq;
        *y = d > 0.0 ? *y * (1.0 / d) : zd{0.0, 0.0};
    }
    __syncthreads();
}

// out_h (rows_h x kk, row-major, precision T) = X_h (rows_h x kc, column-major, global) Y_h
// (kc x kk, column-major with ld kc, LDS) for two products; a thread per (row, 8 columns).
template <typename T>
__device__ void out_gemm2(cx<T>* o0, const zd* X0, int rows0, const zd* Y0, cx<T>* o1, const zd* X1, int rows1,
                          const zd* Y1, int kc, int kk)
{
    constexpr int CH = 8;
    const int nch = (kk + CH - 1) / CH;
    const int n0 = rows0 * nch, ntot = n0 + (Y1 ? rows1 * nch : 0);
    for (int q = threadIdx.x; q < ntot; q += NT) {
        const int h = q >= n0 ? 1 : 0;
        const int qq = q - h * n0, rows = h ? rows1 : rows0;
        const int r = qq % rows, s0 = (qq / rows) * CH;
        const zd* X = h ? X1 : X0;
        const zd* Y = h ? Y1 : Y0;
        zd acc[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) acc[u] = {0.0, 0.0};
        for (int t = 0; t < kc; ++t) {
            const zd x = X[(size_t)t * rows + r];
#pragma unroll
            for (int u = 0; u < CH; ++u)
                if (s0 + u < kk) acc[u] += x * Y[(size_t)(s0 + u) * kc + t];
        }
        cx<T>* out = h ? o1 : o0;
#pragma unroll
        for (int u = 0; u < CH; ++u)
            if (s0 + u < kk) stz(out + (size_t)r * kk + s0 + u, acc[u]);
    }
    __syncthreads();
}

// Recompression of U (3m x kc), V (3n x kc) of the scratch slot w at absolute tolerance tol;
// returns kk > 0 with the factors written over Hout, or 0 (face kept dense).  Scratch:
// G = T_U, VJ = T_V, RU = R_U then B^H then the Vbar coefficients, RV = R_V then the Ubar
// coefficients, M = the pivoted QR.
template <typename T>
__device__ int recompress(cx<T>* Hout, int m, int n, const AcaWork& w, int kc, double tol, Rs& L)
{
    zd* Lm = L.m;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    chol_qr(w.U, 3 * m, kc, w.RU, w.G, L);
    chol_qr(w.V, 3 * n, kc, w.RV, w.VJ, L);
    for (int q = threadIdx.x; q < kc * kc; q += NT) {
        const int i = q % kc, j = q / kc;
        zd s = {0.0, 0.0};
        for (int t = max(i, j); t < kc; ++t) s += mul_conj(w.RU[(size_t)t * kc + i], w.RV[(size_t)t * kc + j]);
        Lm[q] = s;
    }
    __syncthreads();
    double rest2 = 0.0;
    const int kq = qrcp(Lm, kc, QRCP_FRAC * tol, L, &rest2);
    if (kq == 0) return 0;
    // keep the pivoted QR, form B^H (kc x kq): B^H[perm[c]][i] = conj(R[i][c]), i <= c
    for (int q = threadIdx.x; q < kc * kc; q += NT) w.M[q] = Lm[q];
    __syncthreads();
    for (int q = threadIdx.x; q < kc * kq; q += NT) {
        const int c = q % kc, i = q / kc;
        const zd v = i <= c ? conj(w.M[(size_t)c * kc + i]) : zd{0.0, 0.0};
        Lm[(size_t)i * kc + L.perm[c]] = v;
        w.RU[(size_t)i * kc + L.perm[c]] = v;
    }
    __syncthreads();
    if (kq / 2 <= NT / 32) jacobi<32>(Lm, kc, kq, kc, L);
    else jacobi<16>(Lm, kc, kq, kc, L);
    for (int c = wv; c < kq; c += NW) {
        double s = 0.0;
        for (int r = lane; r < kc; r += 64) s += abs2(Lm[(size_t)c * kc + r]);
        s = wsum(s);
        if (lane == 0) L.sv[c] = sqrt(s);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < kq; c += NT) {
        const double sc = L.sv[c];
        int rank = 0;
        for (int c2 = 0; c2 < kq; ++c2) {
            const double s2 = L.sv[c2];
            rank += (s2 > sc || (s2 == sc && c2 < c)) ? 1 : 0;
        }
        L.order[rank] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = rest2;
        for (int c = 0; c < kq; ++c) tot += L.sv[c] * L.sv[c];
        int kk = kq;
        double tail = rest2;
        while (kk > 0) {
            const double s = L.sv[L.order[kk - 1]];
            if (sqrt(tail + s * s) <= tol) {
                tail += s * s;
                --kk;
            } else {
                break;
            }
        }
        if (tot > 0.0 && kk == 0) kk = 1;
        if ((long long)kk * (m + n) >= 3LL * m * n) kk = 0;
        L.piv = kk;
    }
    __syncthreads();
    const int kk = L.piv;
    if (kk <= 0) return 0;
    // Ubar coefficients -> RV: sigma_s [VJ_s; 0] with VJ_s = B W_s / sigma_s^2 (kq entries);
    // Vbar coefficients -> RU: W_s / sigma_s
    for (int q = threadIdx.x; q < kc * kk; q += NT) {
        const int i = q % kc, s = q / kc;
        const int c = L.order[s];
        const double sg = L.sv[c];
        zd v = {0.0, 0.0};
        if (i < kq && sg > 0.0) {
            for (int r = 0; r < kc; ++r) v += conj_mul(w.RU[(size_t)i * kc + r], Lm[(size_t)c * kc + r]);
            v = v * (1.0 / sg);
        }
        w.RV[(size_t)s * kc + i] = v;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kc * kk; q += NT) {
        const int r = q % kc, s = q / kc;
        const int c = L.order[s];
        const double sg = L.sv[c];
        w.RU[(size_t)s * kc + r] = sg > 0.0 ? Lm[(size_t)c * kc + r] * (1.0 / sg) : zd{0.0, 0.0};
    }
    __syncthreads();
    // Lm = [Ubar coefficients | Vbar coefficients] when both fit, else one at a time
    const bool both = 2 * kc * kk <= KF * KF;
    zd* Yu = Lm;
    zd* Yv = both ? Lm + (size_t)kc * kk : nullptr;
    for (int q = threadIdx.x; q < kc * kk; q += NT) {
        Yu[q] = w.RV[q];
        if (both) Yv[q] = w.RU[q];
    }
    __syncthreads();
    // apply Q_M = H_0 ... H_{kq-1} (H = I - tau v v^H) to the Ubar coefficients, one
    // wavefront per column
    for (int jq = kq - 1; jq >= 0; --jq) {
        const zd tj = L.tau[jq];
        const zd* vj = w.M + (size_t)jq * kc;
        for (int s = wv; s < kk; s += NW) {
            zd* y = Yu + (size_t)s * kc;
            double dr = 0.0, di = 0.0;
            for (int r = jq + lane; r < kc; r += 64) {
                const zd t = r == jq ? y[r] : conj_mul(vj[r], y[r]);
                dr += t.re;
                di += t.im;
            }
            dr = wsum(dr);
            di = wsum(di);
            const zd f = tj * zd{dr, di};
            for (int r = jq + lane; r < kc; r += 64) y[r] -= (r == jq ? zd{1.0, 0.0} : vj[r]) * f;
        }
        __syncthreads();
    }
    cx<T>* Ub = Hout;
    cx<T>* Vb = Hout + (size_t)3 * m * kk;
    if (both) {
        backsub2(w.G, Yu, w.VJ, Yv, kc, kk);
        out_gemm2(Ub, w.U, 3 * m, Yu, Vb, w.V, 3 * n, Yv, kc, kk);
    } else {
        backsub2(w.G, Yu, nullptr, nullptr, kc, kk);
        out_gemm2<T>(Ub, w.U, 3 * m, Yu, nullptr, nullptr, 0, nullptr, kc, kk);
        for (int q = threadIdx.x; q < kc * kk; q += NT) Lm[q] = w.RU[q];
        __syncthreads();
        backsub2(w.VJ, Lm, nullptr, nullptr, kc, kk);
        out_gemm2<T>(Vb, w.V, 3 * n, Lm, nullptr, nullptr, 0, nullptr, kc, kk);
    }
    return kk;
}

// one workgroup per listed face (item (block << 8) | d, scratch slot = position in the list)
// after k_face_aca: recompresses the slot's ACA columns and rewrites the face descriptor
__global__ __launch_bounds__(NT) void k_face_recomp(CompressArgs A)
{
    __shared__ Rs L;
    const int item = A.list[blockIdx.x];
    const int b = item >> 8, d = item & 255;
    const BlockIn B = A.blocks[b];
    FaceDesc* fp = A.faces + (size_t)b * A.L + d;
    const FaceDesc f = *fp;
    if (f.kk != 0 || f.sel) return;
    const int m = B.rs, n = B.cs;
    AcaWork w = aca_work(A.scratch + (size_t)blockIdx.x * A.scratch_per_slot, m, n, A.kmax);
    const int kc = w.info[0];
    int kk = 0;
    if (kc > 0 && kc <= KF) {
        const double tol = w.tol[0];
        kk = f.fp32 ? recompress((cx<float>*)(A.pool + f.face_off), m, n, w, kc, tol, L)
                    : recompress((cx<double>*)(A.pool + f.face_off), m, n, w, kc, tol, L);
    }
    if (threadIdx.x == 0) {
        if (kk > 0) {
            fp->kk = kk;
            atomicAdd((unsigned long long*)&A.st[b].aca_cols, (unsigned long long)kc);
        } else {
            atomicAdd(&A.st[b].aca_dense, 1);
        }
    }
}

// the same pass on one given matrix H (after k_aca_matrix): out[0] = ACA columns, out[1] = kk
__global__ __launch_bounds__(NT) void k_aca_matrix_recomp(char* H, int m, int n, int fp32, int kmax,
                                                          double* scratch, int* out)
{
    __shared__ Rs L;
    AcaWork w = aca_work(scratch, m, n, kmax);
    const int kc = out[0];
    int kk = 0;
    if (kc > 0 && kc <= KF) {
        const double tol = w.tol[0];
        kk = fp32 ? recompress((cx<float>*)H, m, n, w, kc, tol, L) : recompress((cx<double>*)H, m, n, w, kc, tol, L);
    }
    if (threadIdx.x == 0) out[1] = kk;
}

}  // namespace

void launch_face_recomp(const CompressArgs& A, hipStream_t st)
{
    if (A.nlist > 0) hipLaunchKernelGGL(k_face_recomp, dim3(A.nlist), dim3(NT), 0, st, A);
    BEM_HIP_TRY(hipGetLastError());
}

void launch_aca_matrix_recomp(char* H, int m, int n, int fp32, int kmax, double* scratch, int* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_aca_matrix_recomp, dim3(1), dim3(NT), 0, st, H, m, n, fp32, kmax, scratch, out);
    BEM_HIP_TRY(hipGetLastError());
}

}  // namespace bem
