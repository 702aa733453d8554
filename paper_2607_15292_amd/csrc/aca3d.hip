// aca3d.hip -- matrix-valued 3D-ACA (Algorithm 1, Sec. 3) on every block of the
// H-matrix partition, one workgroup per block, blocks taken from a work queue.
//
// Per block, step d (0-based here):
//   face    H_d[i,j] = ENTRY(i,j,k_d) - sum_{a<d} H_a[i,j] f_a[k_d]
//           near block: generated densely; far block: matrix-valued ACA on the residual
//           rows/columns + QR/SVD recompression (eq. (ACA)), pivot searched on the
//           reconstruction (Sec. 3.1);
//   pivot   (i_d, j_d) = argmax sigma_3(H_d[i,j]) (eq. (SVD) criterion);
//   fibre   f_d[k] = H_d[i_d,j_d]^{-1} (ENTRY(i_d,j_d,k) - sum_{a<d} H_a[i_d,j_d] f_a[k]);
//   norm    ||C^(d)||^2 += 2 Re sum_{a<d} tr(G_ad F_da) + tr(G_dd F_dd) (eq. (FrobNorm),
//           matrix-valued), G_ad = sum_ij H_a^H H_d, F_da = sum_k f_d f_a^H;
//   stop    ||H_d||_F ||f_d||_F <= eps ||C^(d)||_F (eq. (precision)) -> rank d (pair dropped);
//   next    k_{d+1} = argmax over unused k of sigma_3(f_d[k]).
// A residual face below eps ||C^(d-1)||_F ends the block (converged); a face without a
// regular pivot switches the block to dense storage (one face per frequency with a
// selector fibre), as Sec. 3 prescribes.  Pivots, inverses, norms: FP64.
#include "aca3d.hpp"

#ifdef BEM_PHASE_PROF
#define PROF_T0(v) long long v = (threadIdx.x == 0) ? (long long)__builtin_readcyclecounter() : 0
#define PROF_ADD(A, ph, v) \
    do { if (threadIdx.x == 0) atomicAdd((unsigned long long*)(A).prof + (ph), (unsigned long long)((long long)__builtin_readcyclecounter() - v)); } while (0)
#else
#define PROF_T0(v) (void)0
#define PROF_ADD(A, ph, v) (void)0
#endif

namespace bem {

namespace {

constexpr int WG = 256;
constexpr double PIVOT_RTOL = 1e-14;
constexpr int MAX_FAIL = 8;

__device__ __forceinline__ double wsum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct Lds {
    double red[4 * 24];
    double rv[4];
    int ri[4];
    long long off;
    int qidx;
    int flag;
    int piv;
    double s3;
    zd pinv[9];
    double fnorm, hnorm;
    int nextk;
    unsigned char used[MAX_L];
};

// Sum of N per-thread values over the workgroup; every thread gets the totals.
template <int N>
__device__ __forceinline__ void wg_sum(double (&v)[N], Lds& S)
{
    static_assert(N <= 24, "");
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t < N; ++t) {
        double s = wsum(v[t]);
        if (lane == 0) S.red[w * N + t] = s;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < N; ++t) v[t] = ((S.red[t] + S.red[N + t]) + S.red[2 * N + t]) + S.red[3 * N + t];
    __syncthreads();
}

__device__ __forceinline__ double wg_max(double v, Lds& S)
{
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if (lane == 0) S.rv[w] = v;
    __syncthreads();
    v = fmax(fmax(S.rv[0], S.rv[1]), fmax(S.rv[2], S.rv[3]));
    __syncthreads();
    return v;
}

// argmax with ties to the smallest index; NaN counts as -inf
__device__ __forceinline__ void wg_argmax(double& v, int& idx, Lds& S)
{
    if (!(v == v)) v = -1.0;
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        double ov = __shfl_xor(v, o, 64);
        int oi = __shfl_xor(idx, o, 64);
        if (ov > v || (ov == v && oi < idx)) {
            v = ov;
            idx = oi;
        }
    }
    if (lane == 0) {
        S.rv[w] = v;
        S.ri[w] = idx;
    }
    __syncthreads();
    v = S.rv[0];
    idx = S.ri[0];
    for (int k = 1; k < 4; ++k)
        if (S.rv[k] > v || (S.rv[k] == v && S.ri[k] < idx)) {
            v = S.rv[k];
            idx = S.ri[k];
        }
    __syncthreads();
}

__device__ __forceinline__ long long pool_alloc(const CompressArgs& A, long long bytes)
{
    bytes = (bytes + 255) & ~255LL;
    unsigned long long off = atomicAdd(A.pool_top, (unsigned long long)bytes);
    if (off + (unsigned long long)bytes > A.pool_cap) return -1;
    return (long long)off;
}

template <typename T> __device__ __forceinline__ zd ldz(const cx<T>* p) { return {(double)p->re, (double)p->im}; }
template <typename T> __device__ __forceinline__ void stz(cx<T>* p, zd v) { *p = {(T)v.re, (T)v.im}; }

__device__ __forceinline__ blk ld_blk9(const zd* p)
{
    blk b;
#pragma unroll
    for (int t = 0; t < 9; ++t) b.a[t] = p[t];
    return b;
}

// face block (i, j) of a stored face: dense 3m x 3n row-major (kk == 0) or factors
// Ubar (3m x kk) and Vbar (3n x kk), column-major, in precision T.
template <typename T>
__device__ __forceinline__ blk face_block(const char* pool, const FaceDesc& f, int m, int n, int i, int j)
{
    blk b;
    if (f.kk == 0) {
        const cx<T>* H = (const cx<T>*)(pool + f.face_off);
        size_t ld = 3 * (size_t)n;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) b.a[3 * a + c] = ldz(H + (size_t)(3 * i + a) * ld + 3 * j + c);
        return b;
    }
    const cx<T>* U = (const cx<T>*)(pool + f.face_off);
    const cx<T>* V = U + (size_t)3 * m * f.kk;
    b = blk_zero();
    for (int t = 0; t < f.kk; ++t) {
        zd u[3], v[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            u[a] = ldz(U + (size_t)t * 3 * m + 3 * i + a);
            v[a] = ldz(V + (size_t)t * 3 * n + 3 * j + a);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) b.a[3 * a + c] += mul_conj(u[a], v[c]);
    }
    return b;
}

__device__ __forceinline__ blk fibre_at(const char* pool, const FaceDesc& f, int k)
{
    return ld_blk9((const zd*)(pool + f.fib_off) + (size_t)k * 9);
}

// residual of the 3D approximation at block (i, j), frequency k: E -= sum_{a<d} H_a[i,j] f_a[k]
template <typename T>
__device__ __forceinline__ void sub_residual(blk& E, const CompressArgs& A, const FaceDesc* fd, int d, int m, int n,
                                             int i, int j, int k)
{
    for (int a = 0; a < d; ++a) {
        if (fd[a].sel && fd[a].k != k) continue;
        blk H = face_block<T>(A.pool, fd[a], m, n, i, j);
        blk f = fibre_at(A.pool, fd[a], k);
        blk_mul_sub(E, H, f);
    }
}

// ---------------------------------------------------------------- fibre + norm step
// Shared by near and far blocks once H_d is stored and its pivot block is known.
// Returns (via S): fnorm^2, next k; updates norm2 (all threads) with the new pair.
template <typename T, bool MIXED>
__device__ void fibre_and_norm(const CompressArgs& A, const BlockIn& bi, FaceDesc* fd, int d, int kd, int pi, int pj,
                               double& norm2, double& cross_out, double& tdd_out, Lds& S, long long& nent)
{
    const int L = A.L, m = bi.rs, n = bi.cs;
    zd* f = (zd*)(A.pool + fd[d].fib_off);
    double fn2 = 0.0, best = -1.0;
    int bidx = 0x7fffffff;
    for (int k = threadIdx.x; k < L; k += WG) {
        blk E = entry_dispatch<MIXED>(A.c, A.op, bi.rb + pi, bi.cb + pj, k);
        sub_residual<T>(E, A, fd, d, m, n, pi, pj, k);
        blk Pi;
#pragma unroll
        for (int t = 0; t < 9; ++t) Pi.a[t] = S.pinv[t];
        blk fk = blk_mul(Pi, E);
#pragma unroll
        for (int t = 0; t < 9; ++t) f[(size_t)k * 9 + t] = fk.a[t];
        fn2 += blk_fro2(fk);
        double s3 = S.used[k] ? -1.0 : blk_sigma3(fk);
        if (s3 > best || (s3 == best && k < bidx)) {
            best = s3;
            bidx = k;
        }
    }
    if (threadIdx.x == 0) nent += L;
    double v1[1] = {fn2};
    wg_sum<1>(v1, S);
    fn2 = v1[0];
    wg_argmax(best, bidx, S);
    if (threadIdx.x == 0) {
        S.fnorm = fn2;
        S.nextk = best >= 0.0 ? bidx : -1;
    }
    // cross terms tr(G_ad F_da) for a <= d
    zd cross = {0.0, 0.0}, tdd = {0.0, 0.0};
    for (int a = 0; a <= d; ++a) {
        // F_da = sum_k f_d[k] f_a[k]^H
        double Fv[18];
#pragma unroll
        for (int t = 0; t < 18; ++t) Fv[t] = 0.0;
        const zd* fa = (const zd*)(A.pool + fd[a].fib_off);
        for (int k = threadIdx.x; k < L; k += WG) {
            blk x = ld_blk9(f + (size_t)k * 9), y = ld_blk9(fa + (size_t)k * 9);
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    zd s = {0.0, 0.0};
#pragma unroll
                    for (int q = 0; q < 3; ++q) s += mul_conj(x.a[3 * r + q], y.a[3 * c + q]);
                    Fv[2 * (3 * r + c)] += s.re;
                    Fv[2 * (3 * r + c) + 1] += s.im;
                }
        }
        wg_sum<18>(Fv, S);
        blk F;
#pragma unroll
        for (int t = 0; t < 9; ++t) F.a[t] = {Fv[2 * t], Fv[2 * t + 1]};
        zd tad = {0.0, 0.0};
        if (fd[d].kk == 0 && fd[a].kk == 0) {
            // dense faces: sum_p tr(H_a[p]^H H_d[p] F)
            for (int p = threadIdx.x; p < m * n; p += WG) {
                int i = p / n, j = p - i * n;
                blk Ha = face_block<T>(A.pool, fd[a], m, n, i, j);
                blk Hd = face_block<T>(A.pool, fd[d], m, n, i, j);
                blk HF = blk_mul(Hd, F);
#pragma unroll
                for (int t = 0; t < 9; ++t) tad += conj_mul(Ha.a[t], HF.a[t]);
            }
        } else {
            // factors: tr(X Y), X = Ua^H Ud (ka x kd), Y = Vd^H (I (x) F) Va (kd x ka)
            int ka = fd[a].kk, kd = fd[d].kk;
            const cx<T>* Ua = (const cx<T>*)(A.pool + fd[a].face_off);
            const cx<T>* Va = Ua + (size_t)3 * m * ka;
            const cx<T>* Ud = (const cx<T>*)(A.pool + fd[d].face_off);
            const cx<T>* Vd = Ud + (size_t)3 * m * kd;
            for (int w = threadIdx.x; w < ka * kd; w += WG) {
                int s = w / kd, t = w - s * kd;
                zd X = {0.0, 0.0};
                for (int r = 0; r < 3 * m; ++r) X += conj_mul(ldz(Ua + (size_t)s * 3 * m + r), ldz(Ud + (size_t)t * 3 * m + r));
                zd Y = {0.0, 0.0};
                for (int j = 0; j < n; ++j) {
                    zd va[3], vd[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        va[c] = ldz(Va + (size_t)s * 3 * n + 3 * j + c);
                        vd[c] = ldz(Vd + (size_t)t * 3 * n + 3 * j + c);
                    }
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        zd fv = F.a[3 * c] * va[0] + F.a[3 * c + 1] * va[1] + F.a[3 * c + 2] * va[2];
                        Y += conj_mul(vd[c], fv);
                    }
                }
                tad += X * Y;
            }
        }
        double tv[2] = {tad.re, tad.im};
        wg_sum<2>(tv, S);
        if (a < d) cross += zd{tv[0], tv[1]};
        else tdd = zd{tv[0], tv[1]};
    }
    cross_out = cross.re;
    tdd_out = tdd.re;
    norm2 += 2.0 * cross.re + tdd.re;
}

// ---------------------------------------------------------------- near blocks

template <typename T, bool MIXED>
__device__ void near_face(const CompressArgs& A, const BlockIn& bi, FaceDesc* fd, int d, int k, bool residual,
                          double& s3max, int& pidx, double& fmax2, double& hn2, Lds& S, long long& nent)
{
    const int m = bi.rs, n = bi.cs;
    cx<T>* H = (cx<T>*)(A.pool + fd[d].face_off);
    size_t ld = 3 * (size_t)n;
    double best = -1.0, fm = 0.0, h2 = 0.0;
    int bidx = 0x7fffffff;
    for (int p = threadIdx.x; p < m * n; p += WG) {
        int i = p / n, j = p - i * n;
        blk E = entry_dispatch<MIXED>(A.c, A.op, bi.rb + i, bi.cb + j, k);
        if (residual) sub_residual<T>(E, A, fd, d, m, n, i, j, k);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) stz(H + (size_t)(3 * i + a) * ld + 3 * j + c, E.a[3 * a + c]);
        if (sizeof(T) == 4) {
            // pivot search and norms on the stored (rounded) face
#pragma unroll
            for (int t = 0; t < 9; ++t) E.a[t] = {(double)(float)E.a[t].re, (double)(float)E.a[t].im};
        }
        double e2 = blk_fro2(E);
        h2 += e2;
        fm = fmax(fm, e2);
        double s3 = blk_sigma3(E);
        if (s3 > best || (s3 == best && p < bidx)) {
            best = s3;
            bidx = p;
        }
    }
    if (threadIdx.x == 0) nent += (long long)m * n;
    double v[1] = {h2};
    wg_sum<1>(v, S);
    hn2 = v[0];
    fmax2 = wg_max(fm, S);
    wg_argmax(best, bidx, S);
    s3max = best;
    pidx = bidx;
}

// ---------------------------------------------------------------- far blocks: ACA

struct AcaWork {
    zd *U, *V;        // 3m x kmax, 3n x kmax column-major
    zd *G, *RU, *RV;  // kmax x kmax
    zd *M, *VJ;       // kmax x kmax
    double* dn;       // column norms (kmax) / singular values
    int* usedrow;     // m
    int* order;       // kmax
};

__device__ AcaWork aca_work(double* base, int m, int n, int kmax)
{
    AcaWork w;
    zd* z = (zd*)base;
    w.U = z;
    z += (size_t)3 * m * kmax;
    w.V = z;
    z += (size_t)3 * n * kmax;
    w.G = z;
    z += (size_t)kmax * kmax;
    w.RU = z;
    z += (size_t)kmax * kmax;
    w.RV = z;
    z += (size_t)kmax * kmax;
    w.M = z;
    z += (size_t)kmax * kmax;
    w.VJ = z;
    z += (size_t)kmax * kmax;
    w.dn = (double*)z;
    w.usedrow = (int*)(w.dn + kmax);
    w.order = w.usedrow + m;
    return w;
}

size_t __host__ __device__ aca_work_doubles(int m, int n, int kmax)
{
    return (size_t)2 * (3 * (size_t)m * kmax + 3 * (size_t)n * kmax + 5 * (size_t)kmax * kmax) + kmax +
           (m + kmax + 1) / 2 + 8;
}

// residual of the face at block (i, j): ENTRY - 3D residual - current ACA terms
template <typename T, bool MIXED>
__device__ __forceinline__ blk aca_residual(const CompressArgs& A, const BlockIn& bi, const FaceDesc* fd, int d, int k,
                                            bool residual, const AcaWork& w, int kc, int i, int j)
{
    const int m = bi.rs, n = bi.cs;
    blk E = entry_dispatch<MIXED>(A.c, A.op, bi.rb + i, bi.cb + j, k);
    if (residual) sub_residual<T>(E, A, fd, d, m, n, i, j, k);
    for (int c = 0; c < kc; ++c) {
        zd u[3], v[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            u[a] = w.U[(size_t)c * 3 * m + 3 * i + a];
            v[a] = w.V[(size_t)c * 3 * n + 3 * j + a];
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) E.a[3 * a + b] -= mul_conj(u[a], v[b]);
    }
    return E;
}

// Matrix-valued partial-pivot ACA of the residual face; returns the number of columns.
template <typename T, bool MIXED>
__device__ int far_aca(const CompressArgs& A, const BlockIn& bi, const FaceDesc* fd, int d, int k, bool residual,
                       const AcaWork& w, int kmax, double eps, Lds& S, long long& nent)
{
    const int m = bi.rs, n = bi.cs;
    for (int i = threadIdx.x; i < m; i += WG) w.usedrow[i] = 0;
    __syncthreads();
    int kc = 0, fails = 0, irow = 0;
    double norm2S = 0.0, scale2 = 0.0;
    const int maxsteps = min(min(m, n), kmax / 3);
    while (kc + 3 <= 3 * maxsteps) {
        // residual row irow -> V columns kc..kc+2 (as row^H)
        double best = -1.0, rn2 = 0.0, fm = 0.0;
        int bj = 0x7fffffff;
        for (int j = threadIdx.x; j < n; j += WG) {
            blk E = aca_residual<T, MIXED>(A, bi, fd, d, k, residual, w, kc, irow, j);
#pragma unroll
            for (int y = 0; y < 3; ++y)
#pragma unroll
                for (int x = 0; x < 3; ++x) w.V[(size_t)(kc + y) * 3 * n + 3 * j + x] = conj(E.a[3 * y + x]);
            double e2 = blk_fro2(E);
            rn2 += e2;
            fm = fmax(fm, e2);
            double s3 = blk_sigma3(E);
            if (s3 > best || (s3 == best && j < bj)) {
                best = s3;
                bj = j;
            }
        }
        if (threadIdx.x == 0) {
            nent += n;
            w.usedrow[irow] = 1;
        }
        double v1[1] = {rn2};
        wg_sum<1>(v1, S);
        rn2 = v1[0];
        fm = wg_max(fm, S);
        scale2 = fmax(scale2, fm);
        wg_argmax(best, bj, S);
        if (!(best > PIVOT_RTOL * sqrt(scale2))) {
            if (rn2 <= eps * eps * norm2S) break;
            ++fails;
            // next unused row (smallest index)
            int cand = 0x7fffffff;
            for (int i = threadIdx.x; i < m; i += WG)
                if (!w.usedrow[i] && i < cand) cand = i;
            double cv = cand == 0x7fffffff ? -1.0 : 1.0;
            wg_argmax(cv, cand, S);
            if (cv < 0.0 || fails >= MAX_FAIL) break;
            irow = cand;
            continue;
        }
        fails = 0;
        // pivot inverse
        if (threadIdx.x == 0) {
            blk P;
#pragma unroll
            for (int y = 0; y < 3; ++y)
#pragma unroll
                for (int x = 0; x < 3; ++x) P.a[3 * y + x] = conj(w.V[(size_t)(kc + y) * 3 * n + 3 * bj + x]);
            blk Pi = blk_inv(P);
#pragma unroll
            for (int t = 0; t < 9; ++t) S.pinv[t] = Pi.a[t];
        }
        __syncthreads();
        // residual column bj -> U columns kc..kc+2 = column * P^{-1}
        double best2 = -1.0;
        int bi2 = 0x7fffffff;
        for (int i = threadIdx.x; i < m; i += WG) {
            blk E = aca_residual<T, MIXED>(A, bi, fd, d, k, residual, w, kc, i, bj);
            blk Pi;
#pragma unroll
            for (int t = 0; t < 9; ++t) Pi.a[t] = S.pinv[t];
            blk Un = blk_mul(E, Pi);
#pragma unroll
            for (int y = 0; y < 3; ++y)
#pragma unroll
                for (int x = 0; x < 3; ++x) w.U[(size_t)(kc + x) * 3 * m + 3 * i + y] = Un.a[3 * y + x];
            double s3 = w.usedrow[i] ? -1.0 : blk_sigma3(Un);
            if (s3 > best2 || (s3 == best2 && i < bi2)) {
                best2 = s3;
                bi2 = i;
            }
        }
        if (threadIdx.x == 0) nent += m;
        __syncthreads();
        // norms: ||Un||^2, ||Vn||^2, cross = tr(A1^H A2), A1 = Uold^H Un, A2 = Vold^H Vn,
        // and ||Un Vn^H||^2 = tr((Un^H Un)(Vn^H Vn))
        double acc[2] = {0.0, 0.0};
        for (int q = threadIdx.x; q < 3 * (kc + 3); q += WG) {
            int c = q / 3, x = q - 3 * c;  // column c of the old+new factors against new column x
            zd a1 = {0.0, 0.0}, a2 = {0.0, 0.0};
            for (int r = 0; r < 3 * m; ++r) a1 += conj_mul(w.U[(size_t)c * 3 * m + r], w.U[(size_t)(kc + x) * 3 * m + r]);
            for (int r = 0; r < 3 * n; ++r) a2 += conj_mul(w.V[(size_t)c * 3 * n + r], w.V[(size_t)(kc + x) * 3 * n + r]);
            if (c < kc) {
                zd t = conj_mul(a1, a2);
                acc[0] += t.re;
            } else {
                // new-new Grams: store for the trace below
                w.G[(c - kc) * 3 + x] = a1;
                w.G[9 + (c - kc) * 3 + x] = a2;
            }
        }
        wg_sum<2>(acc, S);
        double cross = acc[0];
        double nn = 0.0, un2 = 0.0, vn2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            un2 += w.G[c * 3 + c].re;
            vn2 += w.G[9 + c * 3 + c].re;
            for (int x = 0; x < 3; ++x) nn += (w.G[c * 3 + x] * w.G[9 + x * 3 + c]).re;
        }
        __syncthreads();
        norm2S += 2.0 * cross + nn;
        kc += 3;
        if (sqrt(un2 * vn2) <= eps * sqrt(fmax(norm2S, 0.0))) break;
        wg_argmax(best2, bi2, S);
        if (best2 < 0.0) break;  // all rows used
        irow = bi2;
    }
    return kc;
}

// Cholesky G = R^H R (R upper, kc x kc, column-major ld = kc) in place of R; dependent
// columns get a zero row in R.
__device__ void wg_cholesky(zd* G, zd* R, int kc, Lds& S)
{
    for (int q = threadIdx.x; q < kc * kc; q += WG) R[q] = {0.0, 0.0};
    __syncthreads();
    for (int k = 0; k < kc; ++k) {
        if (threadIdx.x == 0) {
            double piv = G[(size_t)k * kc + k].re;
            S.s3 = piv > 1e-24 ? sqrt(piv) : 0.0;
        }
        __syncthreads();
        double rkk = S.s3;
        for (int j = k + threadIdx.x; j < kc; j += WG) {
            zd g = G[(size_t)j * kc + k];  // G[k][j]
            R[(size_t)j * kc + k] = (j == k) ? zd{rkk, 0.0} : (rkk > 0.0 ? g * (1.0 / rkk) : zd{0.0, 0.0});
        }
        __syncthreads();
        int rem = kc - k - 1;
        for (int q = threadIdx.x; q < rem * rem; q += WG) {
            int ii = k + 1 + q / rem, jj = k + 1 + q % rem;
            if (ii > jj) continue;
            G[(size_t)jj * kc + ii] -= conj_mul(R[(size_t)ii * kc + k], R[(size_t)jj * kc + k]);
        }
        __syncthreads();
    }
}

// X (rows x kc, column-major) <- X R^{-1} (R upper); zero pivots give zero columns.
__device__ void wg_trsm_right(zd* X, int rows, const zd* R, int kc)
{
    for (int r = threadIdx.x; r < rows; r += WG) {
        for (int j = 0; j < kc; ++j) {
            zd s = X[(size_t)j * rows + r];
            for (int i = 0; i < j; ++i) s -= X[(size_t)i * rows + r] * R[(size_t)j * kc + i];
            double rjj = R[(size_t)j * kc + j].re;
            X[(size_t)j * rows + r] = rjj > 0.0 ? s * (1.0 / rjj) : zd{0.0, 0.0};
        }
    }
    __syncthreads();
}

// G = X^H X (kc x kc column-major, full)
__device__ void wg_gram(const zd* X, int rows, int kc, zd* G)
{
    for (int q = threadIdx.x; q < kc * kc; q += WG) {
        int s = q % kc, t = q / kc;
        if (s > t) continue;
        zd acc = {0.0, 0.0};
        for (int r = 0; r < rows; ++r) acc += conj_mul(X[(size_t)s * rows + r], X[(size_t)t * rows + r]);
        G[(size_t)t * kc + s] = acc;
        G[(size_t)s * kc + t] = conj(acc);
    }
    __syncthreads();
}

// Orthonormalise the columns of X (rows x kc) in place: X = Q R with R (upper) returned in
// Rout; column scaling, then CholeskyQR applied twice.
__device__ void wg_qr(zd* X, int rows, int kc, zd* G, zd* Rtmp, zd* Rout, double* dn, Lds& S)
{
    for (int c = threadIdx.x; c < kc; c += WG) {
        double s = 0.0;
        for (int r = 0; r < rows; ++r) s += abs2(X[(size_t)c * rows + r]);
        dn[c] = sqrt(s);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < rows * kc; q += WG) {
        int c = q / rows;
        X[q] = dn[c] > 0.0 ? X[q] * (1.0 / dn[c]) : zd{0.0, 0.0};
    }
    __syncthreads();
    wg_gram(X, rows, kc, G);
    wg_cholesky(G, Rout, kc, S);
    wg_trsm_right(X, rows, Rout, kc);
    wg_gram(X, rows, kc, G);
    wg_cholesky(G, Rtmp, kc, S);
    wg_trsm_right(X, rows, Rtmp, kc);
    // Rout <- Rtmp * Rout * diag(dn)   (upper triangular product)
    for (int q = threadIdx.x; q < kc * kc; q += WG) {
        int i = q % kc, j = q / kc;
        zd s = {0.0, 0.0};
        if (i <= j)
            for (int t = i; t <= j; ++t) s += Rtmp[(size_t)t * kc + i] * Rout[(size_t)j * kc + t];
        G[q] = s * dn[j];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kc * kc; q += WG) Rout[q] = G[q];
    __syncthreads();
}

// One-sided Jacobi SVD of M (kc x kc, column-major): M VJ = W with orthogonal columns.
// Round-robin ordering; every column pair of a round is handled by a group of JG lanes of
// one wavefront (dot products reduced by lane shuffles within the group).
constexpr int JG = 8;
__device__ void wg_jacobi(zd* M, zd* VJ, int kc, Lds& S)
{
    for (int q = threadIdx.x; q < kc * kc; q += WG) VJ[q] = (q % kc == q / kc) ? zd{1.0, 0.0} : zd{0.0, 0.0};
    __syncthreads();
    const int np = kc + (kc & 1);
    const int g = threadIdx.x / JG, gl = threadIdx.x % JG;
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (threadIdx.x == 0) S.flag = 0;
        __syncthreads();
        for (int rnd = 0; rnd < np - 1; ++rnd) {
            for (int pr = g; pr < np / 2; pr += WG / JG) {
                int p, q;
                if (pr == 0) {
                    p = rnd;
                    q = np - 1;
                } else {
                    p = (rnd + pr) % (np - 1);
                    q = (rnd - pr + np - 1) % (np - 1);
                }
                if (p > q) {
                    int t = p;
                    p = q;
                    q = t;
                }
                if (q >= kc) continue;  // uniform within the group
                zd* mp = M + (size_t)p * kc;
                zd* mq = M + (size_t)q * kc;
                double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
                for (int r = gl; r < kc; r += JG) {
                    al += abs2(mp[r]);
                    be += abs2(mq[r]);
                    zd c = conj_mul(mp[r], mq[r]);
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
                double gabs = sqrt(gr * gr + gi * gi);
                if (!(gabs > 1e-15 * sqrt(al * be)) || gabs == 0.0) continue;
                if (gl == 0) S.flag = 1;
                zd e = {gr / gabs, gi / gabs};  // phase of gamma
                double zeta = (be - al) / (2.0 * gabs);
                double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                zd ce = conj(e);
                zd* vp = VJ + (size_t)p * kc;
                zd* vq = VJ + (size_t)q * kc;
                for (int r = gl; r < kc; r += JG) {
                    zd a = mp[r], b = mq[r] * ce;
                    mp[r] = c * a - s * b;
                    mq[r] = (s * a + c * b) * e;
                    zd va = vp[r], vb = vq[r] * ce;
                    vp[r] = c * va - s * vb;
                    vq[r] = (s * va + c * vb) * e;
                }
            }
            __syncthreads();
        }
        int f = S.flag;
        __syncthreads();
        if (!f) break;
    }
}

// Recompression (eq. (ACA)) of U (3m x kc), V (3n x kc) into pool factors Ubar, Vbar of
// rank kk in precision T; returns kk (0 when everything vanishes).
template <typename T>
__device__ int far_recompress(const CompressArgs& A, const BlockIn& bi, FaceDesc& f, const AcaWork& w, int kc,
                              double eps, Lds& S)
{
    const int m = bi.rs, n = bi.cs;
    wg_qr(w.U, 3 * m, kc, w.G, w.M, w.RU, w.dn, S);
    wg_qr(w.V, 3 * n, kc, w.G, w.M, w.RV, w.dn, S);
    // M = RU RV^H
    for (int q = threadIdx.x; q < kc * kc; q += WG) {
        int i = q % kc, j = q / kc;
        zd s = {0.0, 0.0};
        for (int t = max(i, j); t < kc; ++t) s += mul_conj(w.RU[(size_t)t * kc + i], w.RV[(size_t)t * kc + j]);
        w.M[q] = s;
    }
    __syncthreads();
    wg_jacobi(w.M, w.VJ, kc, S);
    for (int c = threadIdx.x; c < kc; c += WG) {
        double s = 0.0;
        for (int r = 0; r < kc; ++r) s += abs2(w.M[(size_t)c * kc + r]);
        w.dn[c] = sqrt(s);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // order by decreasing singular value (selection; kc is small)
        for (int c = 0; c < kc; ++c) w.order[c] = c;
        for (int a = 0; a < kc; ++a) {
            int bsel = a;
            for (int c = a + 1; c < kc; ++c)
                if (w.dn[w.order[c]] > w.dn[w.order[bsel]]) bsel = c;
            int t = w.order[a];
            w.order[a] = w.order[bsel];
            w.order[bsel] = t;
        }
        double tot = 0.0;
        for (int c = 0; c < kc; ++c) tot += w.dn[c] * w.dn[c];
        int kk = kc;
        double tail = 0.0;
        while (kk > 0) {
            double s = w.dn[w.order[kk - 1]];
            if (sqrt(tail + s * s) <= eps * sqrt(tot)) {
                tail += s * s;
                --kk;
            } else {
                break;
            }
        }
        if (tot > 0.0 && kk == 0) kk = 1;
        S.piv = kk;
        long long off = kk > 0 ? pool_alloc(A, (long long)sizeof(cx<T>) * (3 * (long long)m + 3 * (long long)n) * kk) : 0;
        S.off = off;
    }
    __syncthreads();
    int kk = S.piv;
    long long off = S.off;
    if (off < 0) return -1;
    f.face_off = off;
    f.kk = kk;
    cx<T>* Ub = (cx<T>*)(A.pool + off);
    cx<T>* Vb = Ub + (size_t)3 * m * kk;
    // Ubar[:, s] = QU * M[:, order[s]]  (= QU Uc sigma),  Vbar[:, s] = QV * VJ[:, order[s]]
    for (int q = threadIdx.x; q < 3 * m * kk; q += WG) {
        int r = q % (3 * m), s = q / (3 * m);
        int c = w.order[s];
        zd acc = {0.0, 0.0};
        for (int t = 0; t < kc; ++t) acc += w.U[(size_t)t * 3 * m + r] * w.M[(size_t)c * kc + t];
        stz(Ub + q, acc);
    }
    for (int q = threadIdx.x; q < 3 * n * kk; q += WG) {
        int r = q % (3 * n), s = q / (3 * n);
        int c = w.order[s];
        zd acc = {0.0, 0.0};
        for (int t = 0; t < kc; ++t) acc += w.V[(size_t)t * 3 * n + r] * w.VJ[(size_t)c * kc + t];
        stz(Vb + q, acc);
    }
    __syncthreads();
    return kk;
}

// pivot search on the reconstructed far face
template <typename T>
__device__ void far_scan(const CompressArgs& A, const BlockIn& bi, const FaceDesc& f, double& s3max, int& pidx,
                         double& fmax2, double& hn2, Lds& S)
{
    const int m = bi.rs, n = bi.cs;
    double best = -1.0, fm = 0.0, h2 = 0.0;
    int bidx = 0x7fffffff;
    for (int p = threadIdx.x; p < m * n; p += WG) {
        int i = p / n, j = p - i * n;
        blk H = face_block<T>(A.pool, f, m, n, i, j);
        double e2 = blk_fro2(H);
        h2 += e2;
        fm = fmax(fm, e2);
        double s3 = blk_sigma3(H);
        if (s3 > best || (s3 == best && p < bidx)) {
            best = s3;
            bidx = p;
        }
    }
    double v[1] = {h2};
    wg_sum<1>(v, S);
    hn2 = v[0];
    fmax2 = wg_max(fm, S);
    wg_argmax(best, bidx, S);
    s3max = best;
    pidx = bidx;
}

// ---------------------------------------------------------------- one block

template <typename T, bool MIXED>
__device__ void run_block(const CompressArgs& A, int b, double* scratch, Lds& S)
{
    PROF_T0(tpall);
    const BlockIn bi = A.blocks[b];
    const int m = bi.rs, n = bi.cs, L = A.L;
    const bool far = bi.lowrank != 0;  // faces by per-slice ACA
    const long long fbytes = ((long long)sizeof(cx<T>) * 9 * m * n + 15) & ~15LL;
    FaceDesc* fd = A.faces + (size_t)b * L;
    const double eps = bi.far ? A.eps3d_far : A.eps3d;
    const double eps_aca = A.eps_aca_far;
    const int kmax = A.kmax;
    AcaWork w = aca_work(scratch, m, n, kmax);
    long long nent = 0;
    int aca_cols = 0;
    for (int k = threadIdx.x; k < L; k += WG) S.used[k] = 0;
    __syncthreads();
    double norm2 = 0.0;
    int k = 0, rank = 0, status = 0, fallback = 0;
    for (int d = 0; d < L; ++d) {
        // ---- face H_d at k
        double s3max = -1.0, fmax2 = 0.0, hn2 = 0.0;
        int pidx = 0;
        if (!far) {
            if (threadIdx.x == 0) {
                long long off = pool_alloc(A, fbytes + (long long)sizeof(zd) * 9 * L);
                S.off = off;
            }
            __syncthreads();
            long long off = S.off;
            __syncthreads();
            if (off < 0) {
                status = 2;
                break;
            }
            if (threadIdx.x == 0) {
                fd[d].face_off = off;
                fd[d].fib_off = off + fbytes;
                fd[d].kk = 0;
                fd[d].k = k;
                fd[d].sel = 0;
                fd[d].fp32 = sizeof(T) == 4;
            }
            __syncthreads();
            PROF_T0(tp0);
            near_face<T, MIXED>(A, bi, fd, d, k, true, s3max, pidx, fmax2, hn2, S, nent);
            PROF_ADD(A, 0, tp0);
        } else {
            PROF_T0(tp1);
            int kc = far_aca<T, MIXED>(A, bi, fd, d, k, true, w, kmax, eps_aca, S, nent);
            PROF_ADD(A, 1, tp1);
            if (threadIdx.x == 0) {
                long long off = pool_alloc(A, (long long)sizeof(zd) * 9 * L);
                S.off = off;
            }
            __syncthreads();
            long long foff = S.off;
            __syncthreads();
            if (foff < 0) {
                status = 2;
                break;
            }
            int kk = 0;
            FaceDesc f{0, foff, 0, k, 0, 0};
            if (kc > 0) {
                PROF_T0(tp2);
                kk = far_recompress<T>(A, bi, f, w, kc, eps_aca, S);
                PROF_ADD(A, 2, tp2);
                if (kk < 0) {
                    status = 2;
                    break;
                }
            }
            if (threadIdx.x == 0) {
                fd[d] = f;
                if (kk == 0) fd[d].kk = -1;  // empty face marker (not kept)
            }
            __syncthreads();
            aca_cols = max(aca_cols, kk);
            PROF_T0(tp3);
            if (kk > 0) far_scan<T>(A, bi, fd[d], s3max, pidx, fmax2, hn2, S);
            PROF_ADD(A, 3, tp3);
        }
        // ---- converged residual / no regular pivot
        if (d > 0 && sqrt(hn2) <= eps * sqrt(fmax(norm2, 0.0))) {
            rank = d;
            break;
        }
        if (!(s3max > PIVOT_RTOL * sqrt(fmax2))) {
            fallback = 1;
            break;
        }
        const int pi = pidx / n, pj = pidx - (pidx / n) * n;
        if (threadIdx.x == 0) {
            blk P = face_block<T>(A.pool, fd[d], m, n, pi, pj);
            blk Pi = blk_inv(P);
#pragma unroll
            for (int t = 0; t < 9; ++t) S.pinv[t] = Pi.a[t];
            S.used[k] = 1;
        }
        __syncthreads();
        double cross = 0.0, tdd = 0.0;
        PROF_T0(tp4);
        fibre_and_norm<T, MIXED>(A, bi, fd, d, k, pi, pj, norm2, cross, tdd, S, nent);
        PROF_ADD(A, far ? 5 : 4, tp4);
        double fn2 = S.fnorm;
        int nk = S.nextk;
        __syncthreads();
        if (!(sqrt(hn2 * fn2) > eps * sqrt(fmax(norm2, 0.0)))) {
            rank = d;  // the sub-tolerance pair is dropped
            break;
        }
        rank = d + 1;
        if (nk < 0 || d + 1 == L) break;
        k = nk;
    }
    if (fallback && status == 0) {
        // dense storage: one face per frequency, selector fibres
        for (int kf = 0; kf < L; ++kf) {
            if (!far) {
                if (threadIdx.x == 0) S.off = pool_alloc(A, fbytes + (long long)sizeof(zd) * 9 * L);
                __syncthreads();
                long long off = S.off;
                __syncthreads();
                if (off < 0) {
                    status = 2;
                    break;
                }
                if (threadIdx.x == 0) fd[kf] = FaceDesc{off, off + fbytes, 0, kf, 1, (int)(sizeof(T) == 4)};
                __syncthreads();
                double s3, fm2, h2;
                int pdx;
                near_face<T, MIXED>(A, bi, fd, kf, kf, false, s3, pdx, fm2, h2, S, nent);
            } else {
                int kc = far_aca<T, MIXED>(A, bi, fd, kf, kf, false, w, kmax, eps_aca, S, nent);
                if (threadIdx.x == 0) S.off = pool_alloc(A, (long long)sizeof(zd) * 9 * L);
                __syncthreads();
                long long foff = S.off;
                __syncthreads();
                if (foff < 0) {
                    status = 2;
                    break;
                }
                FaceDesc f{0, foff, 0, kf, 1, 0};
                int kk = 0;
                if (kc > 0) {
                    kk = far_recompress<T>(A, bi, f, w, kc, eps_aca, S);
                    if (kk < 0) {
                        status = 2;
                        break;
                    }
                }
                if (threadIdx.x == 0) {
                    fd[kf] = f;
                    if (kk == 0) fd[kf].kk = -1;
                }
                __syncthreads();
                aca_cols = max(aca_cols, kk);
            }
            // selector fibre
            zd* fb = (zd*)(A.pool + fd[kf].fib_off);
            for (int q = threadIdx.x; q < 9 * L; q += WG) {
                int kq = q / 9, t = q - 9 * kq;
                fb[q] = (kq == kf && (t == 0 || t == 4 || t == 8)) ? zd{1.0, 0.0} : zd{0.0, 0.0};
            }
            __syncthreads();
        }
        rank = status ? 0 : L;
    }
    if (threadIdx.x == 0) {
        BlockOut o;
        o.rank = rank;
        o.fallback = fallback;
        o.status = status;
        o.aca_cols = aca_cols;
        o.entries = nent;
        A.out[b] = o;
        if (status) atomicOr(A.err, status);
    }
    PROF_ADD(A, bi.far ? 7 : 6, tpall);
    __syncthreads();
}

template <typename T, bool MIXED>
__global__ __launch_bounds__(WG) void k_aca3d(CompressArgs A)
{
    __shared__ Lds S;
    double* scratch = A.scratch + (size_t)blockIdx.x * A.scratch_per_slot;
    while (true) {
        if (threadIdx.x == 0) S.qidx = atomicAdd(A.queue, 1);
        __syncthreads();
        int q = S.qidx;
        __syncthreads();
        if (q >= A.nblocks) break;
        int b = A.order[q];
        if (A.blocks[b].far)
            run_block<T, MIXED>(A, b, scratch, S);  // admissible: precision of the far field
        else
            run_block<double, false>(A, b, scratch, S);
    }
}

}  // namespace

size_t aca_scratch_doubles(int mmax, int nmax, int kmax) { return aca_work_doubles(mmax, nmax, kmax); }

void launch_aca3d(const CompressArgs& A, int slots, hipStream_t st)
{
    if (A.mixed)
        hipLaunchKernelGGL((k_aca3d<float, true>), dim3(slots), dim3(WG), 0, st, A);
    else
        hipLaunchKernelGGL((k_aca3d<double, false>), dim3(slots), dim3(WG), 0, st, A);
    BEM_HIP_TRY(hipGetLastError());
}

}  // namespace bem
