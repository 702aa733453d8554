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
//                                            the remaining columns have norm <= tol / 2:
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

constexpr int KF_MAX = 96;      // largest core (ACA columns) of the pass

// The pivoted QR of the core stops once its remaining columns are below QRCP_FRAC tol; the
// SVD truncation of the kept rows then has sqrt(1 - QRCP_FRAC^2) of the tolerance left.  At
// 1/2 (rather than 1/4) the Jacobi SVD works on fewer rows: 7 % less recompression time on the
// 5120-triangle sphere for 0.15 % more ACA rank
constexpr double QRCP_FRAC = 0.5;

// Pairs of the Jacobi SVD whose inner product is below JAC_GMIN tol^2 are left as they are.
constexpr double JAC_GMIN = 1e-6;

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

// Lanes per column in the column updates of the pivoted QR and the reflector application:
// a group's reduction tree and scalar work are replicated over its lanes, so groups are
// narrower than a wavefront.
constexpr int CG = 16;

// sum over the aligned group of CG lanes
__device__ __forceinline__ double gsum(double v)
{
#pragma unroll
    for (int o = CG >> 1; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// 1 / sqrt(x) in FP64 to a few ulp: the hardware reciprocal square root refined by two
// Newton steps (y <- y (3 - x y^2) / 2), for positive normal x
__device__ __forceinline__ double rsqrt_d(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    y = y * (1.5 - 0.5 * x * y * y);
    y = y * (1.5 - 0.5 * x * y * y);
    return y;
}

// orders the LDS accesses of the lanes of one wavefront (no hardware wait is needed: a
// wavefront's LDS instructions complete in order)
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int gx() { return threadIdx.x & 31; }
__device__ __forceinline__ int gy() { return threadIdx.x >> 5; }

// The recompression for one workgroup size NT and largest core KF (ACA columns): the LDS
// working set grows as KF^2, so small cores take a smaller configuration of which several
// workgroups share a compute unit.
template <int NT_, int KF_>
struct Rc {
static constexpr int NT = NT_;     // threads of a recompression workgroup
static constexpr int NW = NT / 64; // its wavefronts
static constexpr int KF = KF_;     // largest core (ACA columns)
static_assert(KF <= KF_MAX && NT % 64 == 0, "");
// LDS matrices use the odd leading dimension kc | 1: with complex128 entries (4 banks each),
// an odd stride keeps the accesses of a row (stride ld) of 8 consecutive lanes in distinct
// banks.
static constexpr int LMS = KF * (KF + 1);

struct Rs {
    zd m[LMS];      // kc x kc working matrix, column-major with ld = kc | 1; Gram staging area
    zd tau[KF];     // reflector coefficients of the pivoted QR
    double sv[KF];  // squared column norms, singular values
    int order[KF];  // singular values by decreasing size
    int perm[KF];   // column order of the pivoted QR
    double du[KF];  // column norms of U and V (1 once applied to the columns themselves)
    double dv[KF];
    double s;
    int piv, flag;
};

// 32 x GY thread grid for the element loops over small matrices
static constexpr int GY = NT / 32;

// Lm = X^H X (kc x kc, full Hermitian, ld) for X (rows x kc, column-major, global).  A
// thread owns up to two 2 x 2 tiles of the upper triangle.  Row chunks of X are staged
// through Lm in two planes (even and odd columns), so that the lanes of a tile row read
// consecutive entries.
static constexpr int GT = ((KF / 2) * (KF / 2 + 1) / 2 + NT - 1) / NT;  // 2 x 2 tiles per thread
static __device__ void gram(const zd* X, int rows, int kc, zd* Lm, int ld)
{
    const int nt = (kc + 1) >> 1, ntri = nt * (nt + 1) / 2;
    const int cr = min(rows, LMS / (2 * nt)), pl = cr * nt;
    int ti[GT], tj[GT];
    bool act[GT];
#pragma unroll
    for (int h = 0; h < GT; ++h) {
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
    zd acc[GT][4];
#pragma unroll
    for (int h = 0; h < GT; ++h)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[h][u] = {0.0, 0.0};
    for (int r0 = 0; r0 < rows; r0 += cr) {
        const int nr = min(cr, rows - r0), tot = nr * 2 * nt;
        __syncthreads();
        for (int q0 = 0; q0 < tot; q0 += 4 * NT) {
            zd v[4];
            int o[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + threadIdx.x + u * NT;
                const int c = q / nr, r = q - c * nr;
                o[u] = q < tot ? (c & 1) * pl + r * nt + (c >> 1) : -1;
                v[u] = q < tot && c < kc ? X[(size_t)c * rows + r0 + r] : zd{0.0, 0.0};
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (o[u] >= 0) Lm[o[u]] = v[u];
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < GT; ++h) {
            if (!act[h]) continue;
            const zd* pa = Lm + ti[h];
            const zd* pb = Lm + tj[h];
            for (int r = 0; r < nr; ++r) {
                const zd a0 = pa[r * nt], a1 = pa[pl + r * nt], b0 = pb[r * nt], b1 = pb[pl + r * nt];
                acc[h][0] += conj_mul(a0, b0);
                acc[h][1] += conj_mul(a0, b1);
                acc[h][2] += conj_mul(a1, b0);
                acc[h][3] += conj_mul(a1, b1);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < GT; ++h) {
        if (!act[h]) continue;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = 2 * ti[h] + (u >> 1), j = 2 * tj[h] + (u & 1);
            if (i < kc && j < kc && i <= j) {
                Lm[(size_t)j * ld + i] = acc[h][u];
                Lm[(size_t)i * ld + j] = conj(acc[h][u]);
            }
        }
    }
    __syncthreads();
}

// Cholesky in place: Lm = R^H R with R upper (upper triangle, the strictly lower part
// zeroed); a pivot without positive mass gives a zero row.  Step k updates the trailing
// matrix from the unscaled row k (divided by the pivot) and scales row k - 1 with the pivot
// read one step earlier.  Returns the smallest pivot (before the square root).
static __device__ double cholesky(zd* Lm, int kc, int ld)
{
    const int tx = gx(), ty = gy();
    double pmin = 1e300, pprev = 0.0;
    for (int k = 0; k < kc; ++k) {
        const double p = Lm[(size_t)k * ld + k].re;
        pmin = fmin(pmin, p);
        if (k > 0) {
            const int kr = k - 1;
            const double rk = pprev > 1e-24 ? sqrt(pprev) : 0.0;
            for (int j = kr + threadIdx.x; j < kc; j += NT) {
                zd* e = Lm + (size_t)j * ld + kr;
                *e = j == kr ? zd{rk, 0.0} : (rk > 0.0 ? *e * (1.0 / rk) : zd{0.0, 0.0});
            }
        }
        if (p > 1e-24) {
            const double ip = 1.0 / p;
            for (int j = k + 1 + ty; j < kc; j += GY) {
                const zd rj = Lm[(size_t)j * ld + k] * ip;
                for (int i = k + 1 + tx; i <= j; i += 32) Lm[(size_t)j * ld + i] -= conj_mul(Lm[(size_t)i * ld + k], rj);
            }
        }
        pprev = p;
        __syncthreads();
    }
    if (threadIdx.x == 0 && kc > 0) Lm[(size_t)(kc - 1) * ld + kc - 1] = {pprev > 1e-24 ? sqrt(pprev) : 0.0, 0.0};
    for (int j = ty; j < kc; j += GY)
        for (int i = j + 1 + tx; i < kc; i += 32) Lm[(size_t)j * ld + i] = {0.0, 0.0};
    __syncthreads();
    return pmin;
}

// X (rows x kc, column-major, global) <- X R^{-1}, R upper in Lm (ld); one row per thread,
// blocks of 8 columns; zero pivots give zero columns.
static __device__ void trsm(zd* X, int rows, const zd* Lm, int kc, int ld)
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
                    if (t < nb) acc[t] -= x * Lm[(size_t)(j0 + t) * ld + i];
            }
#pragma unroll
            for (int t = 0; t < NB; ++t) {
                if (t < nb) {
#pragma unroll
                    for (int u = 0; u < t; ++u) acc[t] -= acc[u] * Lm[(size_t)(j0 + t) * ld + j0 + u];
                    const double d = Lm[(size_t)(j0 + t) * ld + j0 + t].re;
                    acc[t] = d > 0.0 ? acc[t] * (1.0 / d) : zd{0.0, 0.0};
                }
            }
#pragma unroll
            for (int t = 0; t < NB; ++t)
                if (t < nb) X[(size_t)(j0 + t) * rows + r] = acc[t];
        }
    }
    __syncthreads();
}

// CholeskyQR of X (rows x kc) with column scaling, repeated once when the first pass meets a
// pivot below CQ2_PIVOT.  The first pass scales the Gram (D^-1 X^H X D^-1, D the column
// norms, kept in dsc) instead of X.  On return Q = X dsc^-1 T^{-1} with T upper in Tout
// (after two passes X holds X D^{-1} R1^{-1} and dsc is 1) and R = R_fact D in Rout, R_fact
// the triangular factor of X D^{-1}; both kc x kc column-major (ld kc) in global scratch.
static __device__ void chol_qr(zd* X, int rows, int kc, zd* Rout, zd* Tout, double* dsc, Rs& L, int ld)
{
    zd* Lm = L.m;
    const int tx = gx(), ty = gy();
    gram(X, rows, kc, Lm, ld);
    for (int c = threadIdx.x; c < kc; c += NT) {
        const double g = Lm[(size_t)c * ld + c].re;
        dsc[c] = g > 0.0 ? sqrt(g) : 0.0;
    }
    __syncthreads();
    for (int j = ty; j < kc; j += GY)
        for (int i = tx; i < kc; i += 32) {
            const double di = dsc[i], dj = dsc[j];
            zd* e = Lm + (size_t)j * ld + i;
            *e = di > 0.0 && dj > 0.0 ? *e * (1.0 / (di * dj)) : zd{0.0, 0.0};
        }
    __syncthreads();
    const double pmin = cholesky(Lm, kc, ld);
    if (pmin >= CQ2_PIVOT) {
        for (int j = ty; j < kc; j += GY)
            for (int i = tx; i < kc; i += 32) {
                const zd v = Lm[(size_t)j * ld + i];
                Tout[(size_t)j * kc + i] = v;
                Rout[(size_t)j * kc + i] = v * dsc[j];
            }
        __syncthreads();
        return;
    }
    for (int q = threadIdx.x; q < rows * kc; q += NT) {
        const double dc = dsc[q / rows];
        X[q] = dc > 0.0 ? X[q] * (1.0 / dc) : zd{0.0, 0.0};
    }
    __syncthreads();
    trsm(X, rows, Lm, kc, ld);
    for (int j = ty; j < kc; j += GY)
        for (int i = tx; i < kc; i += 32) Tout[(size_t)j * kc + i] = Lm[(size_t)j * ld + i];  // R1 (for now)
    __syncthreads();
    gram(X, rows, kc, Lm, ld);
    cholesky(Lm, kc, ld);
    // Rout = R2 R1 D, then Tout = R2
    for (int j = ty; j < kc; j += GY)
        for (int i = tx; i < kc; i += 32) {
            zd s = {0.0, 0.0};
            for (int t = i; t <= j; ++t) s += Lm[(size_t)t * ld + i] * Tout[(size_t)j * kc + t];
            Rout[(size_t)j * kc + i] = i <= j ? s * dsc[j] : zd{0.0, 0.0};
        }
    __syncthreads();
    for (int j = ty; j < kc; j += GY)
        for (int i = tx; i < kc; i += 32) Tout[(size_t)j * kc + i] = Lm[(size_t)j * ld + i];
    for (int c = threadIdx.x; c < kc; c += NT) dsc[c] = 1.0;
    __syncthreads();
}

// Householder QR with column pivoting of Lm (kc x kc, column-major, ld) in place:
// reflectors H = I - tau v v^H with v[0] = 1 stored below the diagonal, stopped at the first
// step whose remaining columns have Frobenius norm <= delta.  Returns the number of steps;
// tau in L.tau, the column order in L.perm, the remaining squared norm in *rest2.
static __device__ int qrcp(zd* Lm, int kc, int ld, double delta, Rs& L, double* rest2)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int c = threadIdx.x / CG; c < kc; c += NT / CG) {
        const int gl = threadIdx.x % CG;
        double s = 0.0;
        for (int r = gl; r < kc; r += CG) s += abs2(Lm[(size_t)c * ld + r]);
        s = gsum(s);
        if (gl == 0) {
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
                zd* aj = Lm + (size_t)j * ld;
                zd* ap = Lm + (size_t)p * ld;
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
        // apply H^H to the columns j + 1 .. kc - 1 (a group of CG lanes per column), refresh
        // the column norms
        const zd tc = conj(L.tau[j]);
        const zd* aj = Lm + (size_t)j * ld;
        for (int c = j + 1 + threadIdx.x / CG; c < kc; c += NT / CG) {
            const int gl = threadIdx.x % CG;
            zd* ac = Lm + (size_t)c * ld;
            double wr = 0.0, wi = 0.0;
            for (int r = j + gl; r < kc; r += CG) {
                const zd v = r == j ? zd{1.0, 0.0} : aj[r];
                const zd t = conj_mul(v, ac[r]);
                wr += t.re;
                wi += t.im;
            }
            wr = gsum(wr);
            wi = gsum(wi);
            const zd f = tc * zd{wr, wi};
            double s = 0.0;
            for (int r = j + gl; r < kc; r += CG) {
                const zd v = r == j ? zd{1.0, 0.0} : aj[r];
                const zd a = ac[r] - v * f;
                ac[r] = a;
                if (r > j) s += abs2(a);
            }
            s = gsum(s);
            if (gl == 0) L.sv[c] = s;
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
// orthogonal columns, rotations not accumulated.  A group of JG lanes per column pair holds
// the pair in registers; round-robin pair order, one barrier per round.  A pair is rotated
// while |<a, b>| > 1e-12 |a| |b| and |<a, b>| > gmin: below gmin (a small fraction of tol^2)
// the pair's non-orthogonality cannot move the truncation at tol.
static constexpr int JG = 16;
static __device__ int jacobi(zd* Lm, int rows, int ncol, int ld, double gmin, Rs& L)
{
    constexpr int RPL = (KF + JG - 1) / JG;
    const int np = ncol + (ncol & 1);
    const int g = threadIdx.x / JG, gl = threadIdx.x % JG;
    const double gmin2 = gmin * gmin;
    if (ncol < 2) return 0;
    int sweep = 0;
    for (; sweep < 40; ++sweep) {
        if (threadIdx.x == 0) L.flag = 0;
        __syncthreads();
        for (int rnd = 0; rnd < np - 1; ++rnd) {
            for (int pr = g; pr < np / 2; pr += NT / JG) {
                int p, q;
                if (pr == 0) {
                    p = rnd;
                    q = np - 1;
                } else {
                    p = rnd + pr;
                    p -= p >= np - 1 ? np - 1 : 0;
                    q = rnd - pr;
                    q += q < 0 ? np - 1 : 0;
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
                for (int u = 0; u < RPL; ++u) {
                    const int r = gl + JG * u;
                    a[u] = r < rows ? mp[r] : zd{0.0, 0.0};
                    b[u] = r < rows ? mq[r] : zd{0.0, 0.0};
                }
#pragma unroll
                for (int u = 0; u < RPL; ++u) {
                    al += abs2(a[u]);
                    be += abs2(b[u]);
                    const zd c = conj_mul(a[u], b[u]);
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
                const double g2 = gr * gr + gi * gi;
                if (!(g2 > 1e-24 * (al * be)) || !(g2 > gmin2)) continue;
                if (gl == 0) L.flag = 1;
                const double ig = rsqrt_d(g2);
                const zd e = {gr * ig, gi * ig};
                const double zeta = (be - al) * (0.5 * ig);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = rsqrt_d(1.0 + t * t), s = c * t;
                const zd ce = conj(e);
#pragma unroll
                for (int u = 0; u < RPL; ++u) {
                    const int r = gl + JG * u;
                    if (r < rows) {
                        const zd bb = b[u] * ce;
                        mp[r] = c * a[u] - s * bb;
                        mq[r] = (s * a[u] + c * bb) * e;
                    }
                }
            }
            __syncthreads();
        }
        const int f = L.flag;
        __syncthreads();
        if (!f) break;
    }
    return sweep + 1;
}

// Y_h <- D_h^{-1} R_h^{-1} Y_h for up to two systems h (kk columns each, column s at
// Y_h + s ldy, kc rows in LDS), R_h upper (kc x kc, column-major, ld kc, global),
// D_h = diag(d_h) (zero entries and zero pivots give zero rows).  Blocks of BS rows from the
// bottom: a thread per column solves the diagonal block, then the rows above are updated as
// a small GEMM; two barriers per block.
static constexpr int BS = 8;
static __device__ void backsub2(const zd* R0, const double* d0, zd* Y0, const zd* R1, const double* d1, zd* Y1, int kc,
                         int kk, int ldy)
{
    const int nsys = Y1 ? 2 : 1;
    for (int i1 = kc; i1 > 0; i1 -= BS) {
        const int i0 = max(0, i1 - BS), nb = i1 - i0;
        for (int q = threadIdx.x; q < nsys * kk; q += NT) {
            const bool h = q >= kk;
            const zd* R = h ? R1 : R0;
            zd* y = (h ? Y1 : Y0) + (size_t)(h ? q - kk : q) * ldy + i0;
            zd v[BS];
#pragma unroll
            for (int a = 0; a < BS; ++a) v[a] = a < nb ? y[a] : zd{0.0, 0.0};
#pragma unroll
            for (int a = BS - 1; a >= 0; --a) {
                if (a < nb) {
                    const zd* Rc = R + (size_t)(i0 + a) * kc + i0;  // column i0 + a, rows i0 ..
                    const double dg = Rc[a].re;
                    const zd ya = dg > 0.0 ? v[a] * (1.0 / dg) : zd{0.0, 0.0};
                    v[a] = ya;
#pragma unroll
                    for (int b = 0; b < a; ++b) v[b] -= Rc[b] * ya;
                }
            }
#pragma unroll
            for (int a = 0; a < BS; ++a)
                if (a < nb) y[a] = v[a];
        }
        __syncthreads();
        if (i0 == 0) break;
        for (int q = threadIdx.x; q < nsys * i0 * kk; q += NT) {
            const bool h = q >= i0 * kk;
            const int qq = h ? q - i0 * kk : q;
            const int s = qq / i0, t = qq - s * i0;
            const zd* R = h ? R1 : R0;
            zd* y = (h ? Y1 : Y0) + (size_t)s * ldy;
            zd acc = y[t];
#pragma unroll
            for (int a = 0; a < BS; ++a)
                if (a < nb) acc -= R[(size_t)(i0 + a) * kc + t] * y[i0 + a];
            y[t] = acc;
        }
        __syncthreads();
    }
    const int tx = gx(), ty = gy();
    for (int s = ty; s < nsys * kk; s += GY) {
        const bool h = s >= kk;
        const double* d = h ? d1 : d0;
        zd* y = (h ? Y1 : Y0) + (size_t)(h ? s - kk : s) * ldy;
        for (int i = tx; i < kc; i += 32) y[i] = d[i] > 0.0 ? y[i] * (1.0 / d[i]) : zd{0.0, 0.0};
    }
    __syncthreads();
}

// out_h (rows_h x kk, row-major, precision T; CM: column-major complex128) = X_h (rows_h x kc,
// column-major, global) Y_h (kc x kk, column-major with ld ldy, LDS) for up to two products; a
// thread per (row, 8 columns).
template <typename T, bool CM = false>
static __device__ void out_gemm2(cx<T>* o0, const zd* X0, int rows0, const zd* Y0, cx<T>* o1, const zd* X1, int rows1,
                          const zd* Y1, int kc, int kk, int ldy)
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
#pragma unroll 8
        for (int t = 0; t < kc; ++t) {
            const zd x = X[(size_t)t * rows + r];
#pragma unroll
            for (int u = 0; u < CH; ++u)
                if (s0 + u < kk) acc[u] += x * Y[(size_t)(s0 + u) * ldy + t];
        }
        cx<T>* out = h ? o1 : o0;
#pragma unroll
        for (int u = 0; u < CH; ++u)
            if (s0 + u < kk) {
                if (CM) ((zd*)out)[(size_t)(s0 + u) * rows + r] = acc[u];
                else stz(out + (size_t)r * kk + s0 + u, acc[u]);
            }
    }
    __syncthreads();
}

// Recompression of U (3m x kc), V (3n x kc) of the scratch slot w at absolute tolerance tol;
// returns kk > 0 with the factors written over Hout, or 0 (face kept dense).  Scratch:
// G = T_U, VJ = T_V, RU = R_U then B^H then the Vbar coefficients, RV = R_V then the Ubar
// coefficients, M = the pivoted QR (all kc x kc, ld kc).
// Algorithmic flops of the executed parts of one recompression (complex multiply-add = 8):
// stage 0 = QR factors, core and pivoted QR; 1 = + Jacobi; 2 = + coefficients, reflectors,
// back-substitutions and output products.
static __device__ double recomp_flops(int stage, int m, int n, int kc, int kq, int sweeps, int kk)
{
    const double c = kc, ru = 3.0 * m, rv = 3.0 * n;
    double f = 8.0 * ((ru + rv) * c * (c + 1.0) / 2.0 + 2.0 * c * c * c / 6.0 + c * c * c / 3.0);
    for (int j = 0; j < kq; ++j) f += 16.0 * (double)(kc - j) * (double)(kc - j);
    if (stage >= 1) f += 24.0 * sweeps * (double)kq * (kq - 1) / 2.0 * c;
    if (stage >= 2) {
        f += 8.0 * c * c * kk + 8.0 * c * c * kk + 8.0 * (ru + rv) * c * kk;
        for (int j = 0; j < kq; ++j) f += 16.0 * (double)kk * (double)(kc - j);
    }
    return f;
}

// MODE 0: the factors overwrite the face (row-major, precision T) when they take less memory
// than the dense face.  MODE 1 (the intermediate recompression of a run that reached the column
// capacity): the factors go to the slot's other column half (w.U2, w.V2) in complex128
// column-major, at most KF_RESUME of them, with no memory rule.  MODE 2 (a face of the 3D-ACA
// loop): to w.U2, w.V2 as in MODE 1, with the memory rule of MODE 0.  rel > 0: the tolerance
// is at least rel ||U V^H||_F (eq. (ACA) truncated relative to the face's own norm).
static constexpr int KF_RESUME = KF_MAX - 12;
template <typename T, int MODE = 0>
static __device__ int recompress(cx<T>* Hout, int m, int n, const AcaWork& w, int kc, double tol, Rs& L, double& flop,
                                 double rel = 0.0)
{
    constexpr bool CM = MODE != 0;
    zd* Lm = L.m;
    const int ld = kc | 1;
    const int tx = gx(), ty = gy();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    chol_qr(w.U, 3 * m, kc, w.RU, w.G, L.du, L, ld);
    chol_qr(w.V, 3 * n, kc, w.RV, w.VJ, L.dv, L, ld);
    // M = R_U R_V^H
    double m2 = 0.0;
    for (int j = ty; j < kc; j += GY)
        for (int i = tx; i < kc; i += 32) {
            zd s = {0.0, 0.0};
            for (int t = max(i, j); t < kc; ++t) s += mul_conj(w.RU[(size_t)t * kc + i], w.RV[(size_t)t * kc + j]);
            Lm[(size_t)j * ld + i] = s;
            m2 += abs2(s);
        }
    if (rel > 0.0) {
        // ||M||_F = ||U V^H||_F: per-wavefront partial sums in L.sv, then every thread adds them
        m2 = wsum(m2);
        if (lane == 0) L.sv[wv] = m2;
        __syncthreads();
        double tot = 0.0;
        for (int q = 0; q < NW; ++q) tot += L.sv[q];
        tol = fmax(tol, rel * sqrt(tot));
    }
    __syncthreads();
    double rest2 = 0.0;
    const int kq = qrcp(Lm, kc, ld, QRCP_FRAC * tol, L, &rest2);
    flop = recomp_flops(0, m, n, kc, kq, 0, 0);
    if (kq == 0) return 0;
    // keep the pivoted QR, form B^H (kc x kq): B^H[perm[c]][i] = conj(R[i][c]), i <= c
    for (int j = ty; j < kc; j += GY)
        for (int i = tx; i < kc; i += 32) w.M[(size_t)j * kc + i] = Lm[(size_t)j * ld + i];
    __syncthreads();
    for (int i = ty; i < kq; i += GY)
        for (int c = tx; c < kc; c += 32) {
            const zd v = i <= c ? conj(w.M[(size_t)c * kc + i]) : zd{0.0, 0.0};
            Lm[(size_t)i * ld + L.perm[c]] = v;
            w.RU[(size_t)i * kc + L.perm[c]] = v;
        }
    __syncthreads();
    const int sweeps = jacobi(Lm, kc, kq, ld, JAC_GMIN * tol * tol, L);
    flop = recomp_flops(1, m, n, kc, kq, sweeps, 0);
    for (int c = wv; c < kq; c += NW) {
        double s = 0.0;
        for (int r = lane; r < kc; r += 64) s += abs2(Lm[(size_t)c * ld + r]);
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
        if (MODE == 1 ? kk > KF_RESUME : (long long)kk * (m + n) >= 3LL * m * n) kk = 0;
        L.piv = kk;
    }
    __syncthreads();
    const int kk = L.piv;
    if (kk <= 0) return 0;
    flop = recomp_flops(2, m, n, kc, kq, sweeps, kk);
    // Ubar coefficients -> RV: sigma_s [VJ_s; 0] with VJ_s = B W_s / sigma_s^2 (kq entries);
    // Vbar coefficients -> RU: W_s / sigma_s
    for (int s = ty; s < kk; s += GY) {
        const int c = L.order[s];
        const double sg = L.sv[c];
        const zd* Wc = Lm + (size_t)c * ld;
        for (int i = tx; i < kc; i += 32) {
            zd v = {0.0, 0.0};
            if (i < kq && sg > 0.0) {
                const zd* Bi = w.RU + (size_t)i * kc;
                for (int r = 0; r < kc; ++r) v += conj_mul(Bi[r], Wc[r]);
                v = v * (1.0 / sg);
            }
            w.RV[(size_t)s * kc + i] = v;
        }
    }
    __syncthreads();
    for (int s = ty; s < kk; s += GY) {
        const int c = L.order[s];
        const double sg = L.sv[c];
        for (int r = tx; r < kc; r += 32)
            w.RU[(size_t)s * kc + r] = sg > 0.0 ? Lm[(size_t)c * ld + r] * (1.0 / sg) : zd{0.0, 0.0};
    }
    __syncthreads();
    // Lm = [Ubar coefficients | Vbar coefficients] (columns of stride ld) when both fit, else
    // one at a time
    const bool both = 2 * ld * kk <= LMS;
    zd* Yu = Lm;
    zd* Yv = both ? Lm + (size_t)ld * kk : nullptr;
    for (int s = ty; s < kk; s += GY)
        for (int i = tx; i < kc; i += 32) {
            Yu[(size_t)s * ld + i] = w.RV[(size_t)s * kc + i];
            if (both) Yv[(size_t)s * ld + i] = w.RU[(size_t)s * kc + i];
        }
    __syncthreads();
    // apply Q_M = H_0 ... H_{kq-1} (H = I - tau v v^H) to the Ubar coefficients, a group of
    // CG lanes per column
    for (int jq = kq - 1; jq >= 0; --jq) {
        const zd tj = L.tau[jq];
        const zd* vj = w.M + (size_t)jq * kc;
        const int gl = threadIdx.x % CG;
        for (int s = threadIdx.x / CG; s < kk; s += NT / CG) {
            zd* y = Yu + (size_t)s * ld;
            double dr = 0.0, di = 0.0;
            for (int r = jq + gl; r < kc; r += CG) {
                const zd t = r == jq ? y[r] : conj_mul(vj[r], y[r]);
                dr += t.re;
                di += t.im;
            }
            dr = gsum(dr);
            di = gsum(di);
            const zd f = tj * zd{dr, di};
            for (int r = jq + gl; r < kc; r += CG) y[r] -= (r == jq ? zd{1.0, 0.0} : vj[r]) * f;
        }
        __syncthreads();
    }
    cx<T>* Ub = CM ? (cx<T>*)w.U2 : Hout;
    cx<T>* Vb = CM ? (cx<T>*)w.V2 : Hout + (size_t)3 * m * kk;
    if (both) {
        backsub2(w.G, L.du, Yu, w.VJ, L.dv, Yv, kc, kk, ld);
        out_gemm2<T, CM>(Ub, w.U, 3 * m, Yu, Vb, w.V, 3 * n, Yv, kc, kk, ld);
    } else {
        backsub2(w.G, L.du, Yu, nullptr, nullptr, nullptr, kc, kk, ld);
        out_gemm2<T, CM>(Ub, w.U, 3 * m, Yu, nullptr, nullptr, 0, nullptr, kc, kk, ld);
        for (int s = ty; s < kk; s += GY)
            for (int i = tx; i < kc; i += 32) Lm[(size_t)s * ld + i] = w.RU[(size_t)s * kc + i];
        __syncthreads();
        backsub2(w.VJ, L.dv, Lm, nullptr, nullptr, nullptr, kc, kk, ld);
        out_gemm2<T, CM>(Vb, w.V, 3 * n, Lm, nullptr, nullptr, 0, nullptr, kc, kk, ld);
    }
    return kk;
}
};  // struct Rc

using RcBig = Rc<1024, KF_MAX>;  // one workgroup per compute unit (149 KB of LDS)
using RcSmall = Rc<256, 48>;     // 40 KB of LDS: four workgroups per compute unit
constexpr int KC_SMALL = 48;     // cores of at most this many columns take RcSmall

// one workgroup per listed face (item (block << 8) | d, scratch slot = position in the list)
// after k_face_aca: recompresses the slot's ACA columns and rewrites the face descriptor.  A
// run that reached the column capacity (state -2) is recompressed at tol / 4 into the slot's
// other half and left for a resume launch (state -3); every other face ends at state -4.
// Two launches share the list: R = RcSmall takes the faces of 1..KC_SMALL columns, R = RcBig
// (KLO = KC_SMALL) all others, so every face is finished by exactly one of them.
template <class R, int KLO>
__global__ __launch_bounds__(R::NT) void k_face_recomp(CompressArgs A)
{
    constexpr bool BIG = R::KF == KF_MAX;
    __shared__ typename R::Rs L;
    const int item = A.list[blockIdx.x];
    const int b = item >> 8, d = item & 255;
    const BlockIn B = A.blocks[b];
    FaceDesc* fp = A.faces + (size_t)b * A.L + d;
    const FaceDesc f = *fp;
    if (f.kk != 0 || f.sel) return;
    const int m = B.rs, n = B.cs;
    AcaWork w = aca_work(A.scratch + A.slot_off[blockIdx.x], m, n, A.kmax, ACA_HALVES);
    const int kc = w.info[0];
    if (kc == -3 || kc == -4) return;
    if (BIG ? (kc > 0 && kc <= KLO) : !(kc > KLO && kc <= R::KF)) return;
    aca_select_half(w);
    int kk = 0;
    double flop = 0.0;
    if (kc > 0 && kc <= R::KF && A.iloop) {
        kk = R::template recompress<double, 2>(nullptr, m, n, w, kc, 0.0, L, flop, A.eps_aca_far);
    } else if (kc > 0 && kc <= R::KF) {
        const double tol = w.tol[0];
        kk = f.fp32 ? R::recompress((cx<float>*)(A.pool + f.face_off), m, n, w, kc, tol, L, flop)
                    : R::recompress((cx<double>*)(A.pool + f.face_off), m, n, w, kc, tol, L, flop);
    } else if (BIG && kc == -2) {
        kk = R::template recompress<double, 1>(nullptr, m, n, w, w.info[1], 0.25 * w.tol[0], L, flop);
    }
    if (threadIdx.x == 0) {
        atomicAdd(&A.st[b].recomp_flop, flop);
        if (A.iloop) {
            // factors in the slot's other half (k_iloop_store moves them to the pool)
            w.info[1] = kk;
            w.info[2] = kc;
            w.info[0] = kc > 0 && kk > 0 ? -5 : -4;
        } else if (kc == -2 && kk > 0) {
            w.info[1] = kk;
            w.info[3] ^= 1;
            w.info[0] = -3;
            atomicAdd(A.pending, 1);
        } else {
            w.info[0] = -4;
            if (kc > 0 && kk > 0) {
                fp->kk = kk;
                atomicAdd((unsigned long long*)&A.st[b].aca_cols, (unsigned long long)kc);
            } else {
                atomicAdd(&A.st[b].aca_dense, 1);
            }
        }
    }
}

// the same pass on one given matrix H (after k_aca_matrix): out[0] = ACA columns, out[1] = kk
__global__ __launch_bounds__(RcBig::NT) void k_aca_matrix_recomp(char* H, int m, int n, int fp32, int kmax,
                                                                double* scratch, int* out)
{
    using R = RcBig;
    __shared__ R::Rs L;
    AcaWork w = aca_work(scratch, m, n, kmax);
    const int kc = out[0];
    int kk = 0;
    double flop = 0.0;
    if (kc > 0 && kc <= R::KF) {
        const double tol = w.tol[0];
        kk = fp32 ? R::recompress((cx<float>*)H, m, n, w, kc, tol, L, flop)
                  : R::recompress((cx<double>*)H, m, n, w, kc, tol, L, flop);
    }
    if (threadIdx.x == 0) out[1] = kk;
}

}  // namespace

void launch_face_recomp(const CompressArgs& A, hipStream_t st)
{
    if (A.nlist > 0) {
        hipLaunchKernelGGL((k_face_recomp<RcBig, KC_SMALL>), dim3(A.nlist), dim3(RcBig::NT), 0, st, A);
        hipLaunchKernelGGL((k_face_recomp<RcSmall, 0>), dim3(A.nlist), dim3(RcSmall::NT), 0, st, A);
    }
    BEM_HIP_TRY(hipGetLastError());
}

void launch_aca_matrix_recomp(char* H, int m, int n, int fp32, int kmax, double* scratch, int* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_aca_matrix_recomp, dim3(1), dim3(RcBig::NT), 0, st, H, m, n, fp32, kmax, scratch, out);
    BEM_HIP_TRY(hipGetLastError());
}

}  // namespace bem
