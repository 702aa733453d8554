// aca3d.hip -- matrix-valued 3D-ACA (Algorithm 1, Sec. 3) on every block of the
// H-matrix partition, as a pipeline of batched kernels: the host steps the algorithm
// (d = 0, 1, ...) and every phase of a step runs over all blocks still iterating.
//
// Per block, step d:
//   face    H_d[i,j] = ENTRY(i,j,k_d) - sum_{a<d} H_a[i,j] f_a[k_d]
//           dense blocks: every pair generated (k_face_dense, one workgroup per 256 pairs);
//           low-rank blocks: matrix-valued ACA on the residual rows/columns and QR/SVD
//           recompression (eq. (ACA)) (k_aca, one workgroup per block), pivot searched on
//           the reconstruction (k_scan_lr), as Sec. 3.1 describes;
//   pivot   (i_d, j_d) = argmax sigma_3(H_d[i,j]) (criterion of eq. (SVD))      (k_pivot)
//   fibre   f_d[k] = H_d[i_d,j_d]^{-1} (ENTRY(i_d,j_d,k) - sum_{a<d} H_a[i_d,j_d] f_a[k])
//           and F_da = sum_k f_d[k] f_a[k]^H                                   (k_fibre)
//   norm    ||C^(d)||^2 += 2 Re sum_{a<d} tr(G_ad F_da) + tr(G_dd F_dd),
//           G_ad = sum_ij H_a^H H_d (eq. (FrobNorm), matrix-valued)   (k_cross_*, k_final)
//   stop    ||H_d||_F ||f_d||_F <= eps ||C^(d)||_F (eq. (precision)) -> rank d (pair dropped);
//   next    k_{d+1} = argmax over unused k of sigma_3(f_d[k]).
// A residual face below eps ||C^(d-1)||_F ends the block (converged); a face without a
// regular pivot switches the block to dense storage (one face per frequency with a
// selector fibre), as Sec. 3 prescribes.  Pivots, inverses and norms are FP64.
#include "aca3d.hpp"

namespace bem {

namespace {

constexpr int WG = 256;
constexpr double PIVOT_RTOL = 1e-14;
constexpr int MAX_FAIL = 8;

// ---------------------------------------------------------------- workgroup reductions

struct Red {
    double red[4 * 24];
    double rv[4];
    int ri[4];
};

__device__ __forceinline__ double wsum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int N>
__device__ __forceinline__ void wg_sum(double (&v)[N], Red& S)
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

__device__ __forceinline__ double wg_max(double v, Red& S)
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
__device__ __forceinline__ void wg_argmax(double& v, int& idx, Red& S)
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

// ---------------------------------------------------------------- storage helpers

__device__ __forceinline__ long long pool_alloc(const CompressArgs& A, long long bytes)
{
    bytes = (bytes + 255) & ~255LL;
    unsigned long long off = atomicAdd(A.pool_top, (unsigned long long)bytes);
    if (off + (unsigned long long)bytes > A.pool_cap) {
        atomicOr(A.err, 2);
        return -1;
    }
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

template <typename T>
__device__ __forceinline__ blk lowrank_block(const char* pool, const FaceDesc& f, int m, int i, int j)
{
    const int kk = f.kk;
    const cx<T>* U = (const cx<T>*)(pool + f.face_off) + (size_t)(3 * i) * kk;
    const cx<T>* V = (const cx<T>*)(pool + f.face_off) + (size_t)3 * m * kk + (size_t)(3 * j) * kk;
    blk b = blk_zero();
    for (int t = 0; t < kk; ++t) {
        zd u[3], v[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            u[a] = ldz(U + (size_t)a * kk + t);
            v[a] = ldz(V + (size_t)a * kk + t);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) b.a[3 * a + c] += mul_conj(u[a], v[c]);
    }
    return b;
}

// block (i, j) of a stored face
__device__ __forceinline__ blk face_block(const char* pool, const FaceDesc& f, int m, int n, int i, int j)
{
    blk b;
    if (f.kk == 0) {
        size_t ld = 3 * (size_t)n;
        if (f.fp32) {
            const zf* H = (const zf*)(pool + f.face_off);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) b.a[3 * a + c] = ldz(H + (size_t)(3 * i + a) * ld + 3 * j + c);
        } else {
            const zd* H = (const zd*)(pool + f.face_off);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) b.a[3 * a + c] = H[(size_t)(3 * i + a) * ld + 3 * j + c];
        }
        return b;
    }
    if (f.kk < 0) return blk_zero();
    return f.fp32 ? lowrank_block<float>(pool, f, m, i, j) : lowrank_block<double>(pool, f, m, i, j);
}

__device__ __forceinline__ blk fibre_at(const char* pool, const FaceDesc& f, int k)
{
    return ld_blk9((const zd*)(pool + f.fib_off) + (size_t)k * 9);
}

// E -= sum_{a<d} H_a[i,j] f_a[k]   (the 3D approximation C^(d-1) at (i, j, k))
__device__ __forceinline__ void sub_residual(blk& E, const CompressArgs& A, const FaceDesc* fd, int d, int m, int n,
                                             int i, int j, int k)
{
    for (int a = 0; a < d; ++a) {
        const FaceDesc f = fd[a];
        if (f.sel && f.k != k) continue;
        blk H = face_block(A.pool, f, m, n, i, j);
        blk fk = fibre_at(A.pool, f, k);
        blk_mul_sub(E, H, fk);
    }
}

__device__ __forceinline__ blk entry_of(const CompressArgs& A, const BlockIn& B, int i, int j, int k)
{
    if (A.mixed && B.far) return entry_dispatch<true>(A.c, A.op, B.rb + i, B.cb + j, k);
    return entry_dispatch<false>(A.c, A.op, B.rb + i, B.cb + j, k);
}

__device__ __forceinline__ double block_eps(const CompressArgs& A, const BlockIn& B)
{
    return B.far ? A.eps3d_far : A.eps3d;
}

__device__ __forceinline__ long long dense_face_bytes(const CompressArgs& A, const BlockIn& B)
{
    size_t zs = (A.mixed && B.far) ? sizeof(zf) : sizeof(zd);
    return ((long long)zs * 9 * B.rs * B.cs + 15) & ~15LL;
}

// Reserve the storage of step d of block b: dense face + fibre, or the fibre of a low-rank
// face (its factors are reserved when their rank is known).  False on pool overflow.
__device__ bool alloc_step(const CompressArgs& A, int b, int d, int k)
{
    const BlockIn B = A.blocks[b];
    FaceDesc f;
    f.k = k;
    f.sel = 0;
    if (!B.lowrank) {
        long long fb = dense_face_bytes(A, B);
        long long off = pool_alloc(A, fb + (long long)sizeof(zd) * 9 * A.L);
        if (off < 0) return false;
        f.face_off = off;
        f.fib_off = off + fb;
        f.kk = 0;
        f.fp32 = (A.mixed && B.far) ? 1 : 0;
    } else {
        long long off = pool_alloc(A, (long long)sizeof(zd) * 9 * A.L);
        if (off < 0) return false;
        f.face_off = 0;
        f.fib_off = off;
        f.kk = -1;
        f.fp32 = A.mixed ? 1 : 0;
    }
    A.faces[(size_t)b * A.L + d] = f;
    return true;
}

// ---------------------------------------------------------------- init

__global__ __launch_bounds__(256) void k_init(CompressArgs A)
{
    int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= A.nblocks) return;
    BlockState s;
    s.k = 0;
    s.rank = 0;
    s.active = 1;
    s.fallback = 0;
    s.stop = 0;
    s.piv = 0;
    s.nextk = -1;
    s.kc = 0;
    s.aca_max = 0;
    s.pad = 0;
    s.norm2 = 0.0;
    s.hn2 = s.fmax2 = s.s3max = s.fn2 = 0.0;
    s.entries = 0;
    for (int t = 0; t < 9; ++t) s.pinv[t] = {0.0, 0.0};
    for (int k = 0; k < A.L; ++k) A.used[(size_t)b * A.L + k] = 0;
    if (!alloc_step(A, b, 0, 0)) s.active = 0;
    A.st[b] = s;
}

// ---------------------------------------------------------------- dense faces

// tile partials: [0] sigma_3 max, [1] pivot pair, [2] sum |H|^2, [3] max block |H|^2,
//                [4] cross re, [5] t_dd re
__global__ __launch_bounds__(WG) void k_face_dense(CompressArgs A)
{
    __shared__ Red S;
    const int item = A.list[blockIdx.x];
    const int b = item >> 12, t = item & 4095;
    if (!A.st[b].active) return;
    const BlockIn B = A.blocks[b];
    const int m = B.rs, n = B.cs, d = A.d;
    const int k = A.st[b].k;
    const FaceDesc* fd = A.faces + (size_t)b * A.L;
    const FaceDesc F = fd[d];
    const int p = t * TILE + threadIdx.x;
    double s3 = -1.0, e2 = 0.0;
    int pi = 0x7fffffff;
    if (p < m * n) {
        const int i = p / n, j = p - (p / n) * n;
        blk E = entry_of(A, B, i, j, k);
        sub_residual(E, A, fd, d, m, n, i, j, k);
        size_t ld = 3 * (size_t)n;
        if (F.fp32) {
            zf* H = (zf*)(A.pool + F.face_off);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    zd v = E.a[3 * a + c];
                    zf w = {(float)v.re, (float)v.im};
                    H[(size_t)(3 * i + a) * ld + 3 * j + c] = w;
                    E.a[3 * a + c] = {(double)w.re, (double)w.im};  // search on the stored face
                }
        } else {
            zd* H = (zd*)(A.pool + F.face_off);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) H[(size_t)(3 * i + a) * ld + 3 * j + c] = E.a[3 * a + c];
        }
        e2 = blk_fro2(E);
        s3 = blk_sigma3(E);
        pi = p;
    }
    double v[1] = {e2};
    wg_sum<1>(v, S);
    double fm = wg_max(e2, S);
    wg_argmax(s3, pi, S);
    if (threadIdx.x == 0) {
        double* tp = A.tp + (size_t)(B.tile0 + t) * 8;
        tp[0] = s3;
        tp[1] = (double)pi;
        tp[2] = v[0];
        tp[3] = fm;
        int cnt = min(TILE, m * n - t * TILE);
        atomicAdd((unsigned long long*)&A.st[b].entries, (unsigned long long)cnt);
    }
}

// ---------------------------------------------------------------- low-rank faces: ACA

struct AcaWork {
    zd *U, *V;        // 3m x kmax, 3n x kmax column-major
    zd *G, *RU, *RV;  // kmax x kmax
    zd *M, *VJ;       // kmax x kmax
    double* dn;       // kmax
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

struct AcaShared {
    Red r;
    zd pinv[9];
    double s;
    long long off;
    int piv, flag;
};

// residual of the face at block (i, j): ENTRY - C^(d-1) - current ACA terms
__device__ __forceinline__ blk aca_residual(const CompressArgs& A, const BlockIn& B, const FaceDesc* fd, int d, int k,
                                            const AcaWork& w, int kc, int i, int j)
{
    const int m = B.rs, n = B.cs;
    blk E = entry_of(A, B, i, j, k);
    sub_residual(E, A, fd, d, m, n, i, j, k);
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
            for (int bb = 0; bb < 3; ++bb) E.a[3 * a + bb] -= mul_conj(u[a], v[bb]);
    }
    return E;
}

// Matrix-valued partial-pivot ACA of the residual face; returns the number of columns.
__device__ int far_aca(const CompressArgs& A, const BlockIn& B, const FaceDesc* fd, int d, int k, const AcaWork& w,
                       int kmax, double eps, AcaShared& S, long long& nent)
{
    const int m = B.rs, n = B.cs;
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
            blk E = aca_residual(A, B, fd, d, k, w, kc, irow, j);
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
        wg_sum<1>(v1, S.r);
        rn2 = v1[0];
        fm = wg_max(fm, S.r);
        scale2 = fmax(scale2, fm);
        wg_argmax(best, bj, S.r);
        if (!(best > PIVOT_RTOL * sqrt(scale2))) {
            if (rn2 <= eps * eps * norm2S) break;
            ++fails;
            int cand = 0x7fffffff;
            for (int i = threadIdx.x; i < m; i += WG)
                if (!w.usedrow[i] && i < cand) cand = i;
            double cv = cand == 0x7fffffff ? -1.0 : 1.0;
            wg_argmax(cv, cand, S.r);
            if (cv < 0.0 || fails >= MAX_FAIL) break;
            irow = cand;
            continue;
        }
        fails = 0;
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
            blk E = aca_residual(A, B, fd, d, k, w, kc, i, bj);
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
        // ||S_k||^2 update: cross = tr(A1^H A2), A1 = Uold^H Un, A2 = Vold^H Vn, and
        // ||Un Vn^H||^2 = tr((Un^H Un)(Vn^H Vn)); one wavefront per (column, new column)
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        double acc = 0.0;
        for (int q = wv; q < 3 * (kc + 3); q += WG / 64) {
            int c = q / 3, x = q - 3 * c;
            double r1 = 0.0, i1 = 0.0, r2 = 0.0, i2 = 0.0;
            for (int r = lane; r < 3 * m; r += 64) {
                zd t = conj_mul(w.U[(size_t)c * 3 * m + r], w.U[(size_t)(kc + x) * 3 * m + r]);
                r1 += t.re;
                i1 += t.im;
            }
            for (int r = lane; r < 3 * n; r += 64) {
                zd t = conj_mul(w.V[(size_t)c * 3 * n + r], w.V[(size_t)(kc + x) * 3 * n + r]);
                r2 += t.re;
                i2 += t.im;
            }
            r1 = wsum(r1);
            i1 = wsum(i1);
            r2 = wsum(r2);
            i2 = wsum(i2);
            zd a1 = {r1, i1}, a2 = {r2, i2};
            if (c < kc) {
                if (lane == 0) acc += conj_mul(a1, a2).re;
            } else if (lane == 0) {
                w.G[(c - kc) * 3 + x] = a1;
                w.G[9 + (c - kc) * 3 + x] = a2;
            }
        }
        double accv[1] = {acc};
        wg_sum<1>(accv, S.r);
        double cross = accv[0];
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
        wg_argmax(best2, bi2, S.r);
        if (best2 < 0.0) break;  // all rows used
        irow = bi2;
    }
    return kc;
}

// Cholesky G = R^H R (R upper, column-major ld = kc); dependent columns get a zero row.
__device__ void wg_cholesky(zd* G, zd* R, int kc, AcaShared& S)
{
    for (int q = threadIdx.x; q < kc * kc; q += WG) R[q] = {0.0, 0.0};
    __syncthreads();
    for (int k = 0; k < kc; ++k) {
        if (threadIdx.x == 0) {
            double piv = G[(size_t)k * kc + k].re;
            S.s = piv > 1e-24 ? sqrt(piv) : 0.0;
        }
        __syncthreads();
        double rkk = S.s;
        for (int j = k + threadIdx.x; j < kc; j += WG) {
            zd g = G[(size_t)j * kc + k];
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

// X (rows x kc, column-major) <- X R^{-1}; zero pivots give zero columns.
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

// G = X^H X (kc x kc column-major, full); one wavefront per column pair, lanes over rows.
__device__ void wg_gram(const zd* X, int rows, int kc, zd* G)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int q = wv; q < kc * kc; q += WG / 64) {
        int s = q % kc, t = q / kc;
        if (s > t) continue;  // uniform per wavefront
        double re = 0.0, im = 0.0;
        for (int r = lane; r < rows; r += 64) {
            zd c = conj_mul(X[(size_t)s * rows + r], X[(size_t)t * rows + r]);
            re += c.re;
            im += c.im;
        }
        re = wsum(re);
        im = wsum(im);
        if (lane == 0) {
            G[(size_t)t * kc + s] = {re, im};
            G[(size_t)s * kc + t] = {re, -im};
        }
    }
    __syncthreads();
}

// X = Q R (R upper in Rout): column scaling, then CholeskyQR applied twice.
__device__ void wg_qr(zd* X, int rows, int kc, zd* G, zd* Rtmp, zd* Rout, double* dn, AcaShared& S)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int c = wv; c < kc; c += WG / 64) {
        double s = 0.0;
        for (int r = lane; r < rows; r += 64) s += abs2(X[(size_t)c * rows + r]);
        s = wsum(s);
        if (lane == 0) dn[c] = sqrt(s);
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
// Round-robin ordering; each column pair of a round is handled by JG lanes of one wavefront.
constexpr int JG = 8;
__device__ void wg_jacobi(zd* M, zd* VJ, int kc, AcaShared& S)
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
                if (q >= kc) continue;  // uniform within the lane group
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
                zd e = {gr / gabs, gi / gabs};
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

// Recompression (eq. (ACA)) of U (3m x kc), V (3n x kc) into row-major pool factors
// Ubar = QU Uc Sigma, Vbar = QV Vc of rank kk (precision T); returns kk, -1 on overflow.
template <typename T>
__device__ int far_recompress(const CompressArgs& A, const BlockIn& B, FaceDesc& f, const AcaWork& w, int kc,
                              double eps, AcaShared& S)
{
    const int m = B.rs, n = B.cs;
    wg_qr(w.U, 3 * m, kc, w.G, w.M, w.RU, w.dn, S);
    wg_qr(w.V, 3 * n, kc, w.G, w.M, w.RV, w.dn, S);
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
        S.off = kk > 0 ? pool_alloc(A, (long long)sizeof(cx<T>) * (3 * (long long)m + 3 * (long long)n) * kk) : 0;
    }
    __syncthreads();
    const int kk = S.piv;
    const long long off = S.off;
    if (off < 0) return -1;
    f.face_off = off;
    f.kk = kk;
    cx<T>* Ub = (cx<T>*)(A.pool + off);
    cx<T>* Vb = Ub + (size_t)3 * m * kk;
    for (int q = threadIdx.x; q < 3 * m * kk; q += WG) {
        int r = q / kk, s = q - r * kk;
        int c = w.order[s];
        zd acc = {0.0, 0.0};
        for (int t = 0; t < kc; ++t) acc += w.U[(size_t)t * 3 * m + r] * w.M[(size_t)c * kc + t];
        stz(Ub + q, acc);
    }
    for (int q = threadIdx.x; q < 3 * n * kk; q += WG) {
        int r = q / kk, s = q - r * kk;
        int c = w.order[s];
        zd acc = {0.0, 0.0};
        for (int t = 0; t < kc; ++t) acc += w.V[(size_t)t * 3 * n + r] * w.VJ[(size_t)c * kc + t];
        stz(Vb + q, acc);
    }
    __syncthreads();
    return kk;
}

// one workgroup per low-rank block of the list (scratch slot = position in the list)
__global__ __launch_bounds__(WG) void k_aca(CompressArgs A)
{
    __shared__ AcaShared S;
    const int b = A.list[blockIdx.x];
    if (!A.st[b].active) return;
    const BlockIn B = A.blocks[b];
    const int d = A.d, k = A.st[b].k;
    FaceDesc* fd = A.faces + (size_t)b * A.L;
    AcaWork w = aca_work(A.scratch + (size_t)blockIdx.x * A.scratch_per_slot, B.rs, B.cs, A.kmax);
    long long nent = 0;
    const double eps = A.eps_aca_far;
    int kc = far_aca(A, B, fd, d, k, w, A.kmax, eps, S, nent);
    FaceDesc f = fd[d];
    int kk = 0;
    if (kc > 0) kk = A.mixed ? far_recompress<float>(A, B, f, w, kc, eps, S) : far_recompress<double>(A, B, f, w, kc, eps, S);
    if (threadIdx.x == 0) {
        if (kk < 0) {
            A.st[b].active = 0;
        } else {
            f.kk = kk > 0 ? kk : -1;
            f.fp32 = A.mixed ? 1 : 0;
            fd[d] = f;
        }
        A.st[b].kc = kc;
        atomicAdd((unsigned long long*)&A.st[b].entries, (unsigned long long)nent);
    }
}

// pivot search on the reconstructed low-rank face (one workgroup per tile)
__global__ __launch_bounds__(WG) void k_scan_lr(CompressArgs A)
{
    __shared__ Red S;
    const int item = A.list[blockIdx.x];
    const int b = item >> 12, t = item & 4095;
    if (!A.st[b].active) return;
    const BlockIn B = A.blocks[b];
    const int m = B.rs, n = B.cs;
    const FaceDesc F = A.faces[(size_t)b * A.L + A.d];
    const int p = t * TILE + threadIdx.x;
    double s3 = -1.0, e2 = 0.0;
    int pi = 0x7fffffff;
    if (p < m * n && F.kk > 0) {
        const int i = p / n, j = p - (p / n) * n;
        blk H = face_block(A.pool, F, m, n, i, j);
        e2 = blk_fro2(H);
        s3 = blk_sigma3(H);
        pi = p;
    }
    double v[1] = {e2};
    wg_sum<1>(v, S);
    double fm = wg_max(e2, S);
    wg_argmax(s3, pi, S);
    if (threadIdx.x == 0) {
        double* tp = A.tp + (size_t)(B.tile0 + t) * 8;
        tp[0] = s3;
        tp[1] = (double)pi;
        tp[2] = v[0];
        tp[3] = fm;
    }
}

// ---------------------------------------------------------------- pivot

__global__ __launch_bounds__(64) void k_pivot(CompressArgs A)
{
    int q = blockIdx.x * 64 + threadIdx.x;
    if (q >= A.nlist) return;
    const int b = A.list[q];
    BlockState s = A.st[b];
    if (!s.active) return;
    const BlockIn B = A.blocks[b];
    const int d = A.d;
    double best = -1.0, h2 = 0.0, fm = 0.0;
    int pi = 0x7fffffff;
    for (int t = 0; t < B.ntile; ++t) {
        const double* tp = A.tp + (size_t)(B.tile0 + t) * 8;
        double v = tp[0];
        int ix = (int)tp[1];
        if (!(v == v)) v = -1.0;
        if (v > best || (v == best && ix < pi)) {
            best = v;
            pi = ix;
        }
        h2 += tp[2];
        fm = fmax(fm, tp[3]);
    }
    s.hn2 = h2;
    s.fmax2 = fm;
    s.s3max = best;
    s.stop = 0;
    const double eps = block_eps(A, B);
    if (d > 0 && sqrt(h2) <= eps * sqrt(fmax(s.norm2, 0.0))) {
        // the residual face vanishes: C^(d-1) reproduces the array; rank d
        s.stop = 1;
        s.active = 0;
        s.rank = d;
    } else if (!(best > PIVOT_RTOL * sqrt(fm))) {
        s.stop = 1;
        s.active = 0;
        s.fallback = 1;
    } else {
        s.piv = pi;
        const int n = B.cs;
        blk P = face_block(A.pool, A.faces[(size_t)b * A.L + d], B.rs, n, pi / n, pi - (pi / n) * n);
        blk Pi = blk_inv(P);
        for (int t = 0; t < 9; ++t) s.pinv[t] = Pi.a[t];
        A.used[(size_t)b * A.L + s.k] = 1;
    }
    A.st[b] = s;
}

// ---------------------------------------------------------------- fibres

__global__ __launch_bounds__(WG) void k_fibre(CompressArgs A)
{
    __shared__ Red S;
    __shared__ zd Pi_s[9];
    const int b = A.list[blockIdx.x];
    if (!A.st[b].active || A.st[b].stop) return;
    const BlockIn B = A.blocks[b];
    const int m = B.rs, n = B.cs, d = A.d, L = A.L;
    const FaceDesc* fd = A.faces + (size_t)b * L;
    const int piv = A.st[b].piv;
    const int pi = piv / n, pj = piv - (piv / n) * n;
    if (threadIdx.x < 9) Pi_s[threadIdx.x] = A.st[b].pinv[threadIdx.x];
    __syncthreads();
    zd* f = (zd*)(A.pool + fd[d].fib_off);
    double fn2 = 0.0, best = -1.0;
    int bk = 0x7fffffff;
    for (int k = threadIdx.x; k < L; k += WG) {
        blk E = entry_of(A, B, pi, pj, k);
        sub_residual(E, A, fd, d, m, n, pi, pj, k);
        blk Pi;
#pragma unroll
        for (int t = 0; t < 9; ++t) Pi.a[t] = Pi_s[t];
        blk fk = blk_mul(Pi, E);
#pragma unroll
        for (int t = 0; t < 9; ++t) f[(size_t)k * 9 + t] = fk.a[t];
        fn2 += blk_fro2(fk);
        double s3 = A.used[(size_t)b * L + k] ? -1.0 : blk_sigma3(fk);
        if (s3 > best || (s3 == best && k < bk)) {
            best = s3;
            bk = k;
        }
    }
    double v1[1] = {fn2};
    wg_sum<1>(v1, S);
    wg_argmax(best, bk, S);
    // F_da = sum_k f_d[k] f_a[k]^H for a <= d
    for (int a = 0; a <= d; ++a) {
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
        if (threadIdx.x == 0)
            for (int t = 0; t < 9; ++t) A.Fda[((size_t)b * L + a) * 9 + t] = {Fv[2 * t], Fv[2 * t + 1]};
    }
    if (threadIdx.x == 0) {
        A.st[b].fn2 = v1[0];
        A.st[b].nextk = best >= 0.0 ? bk : -1;
        atomicAdd((unsigned long long*)&A.st[b].entries, (unsigned long long)L);
    }
}

// ---------------------------------------------------------------- norm cross terms

// dense faces: sum_p tr(H_a[p]^H H_d[p] F_da) for a < d and a = d (one workgroup per tile)
__global__ __launch_bounds__(WG) void k_cross_dense(CompressArgs A)
{
    __shared__ Red S;
    __shared__ zd Fs[MAX_L * 9];
    const int item = A.list[blockIdx.x];
    const int b = item >> 12, t = item & 4095;
    if (!A.st[b].active || A.st[b].stop) return;
    const BlockIn B = A.blocks[b];
    const int m = B.rs, n = B.cs, d = A.d, L = A.L;
    const FaceDesc* fd = A.faces + (size_t)b * L;
    for (int q = threadIdx.x; q < 9 * (d + 1); q += WG) Fs[q] = A.Fda[(size_t)b * L * 9 + q];
    __syncthreads();
    const int p = t * TILE + threadIdx.x;
    zd cross = {0.0, 0.0}, tdd = {0.0, 0.0};
    if (p < m * n) {
        const int i = p / n, j = p - (p / n) * n;
        blk Hd = face_block(A.pool, fd[d], m, n, i, j);
        for (int a = 0; a <= d; ++a) {
            blk F;
#pragma unroll
            for (int q = 0; q < 9; ++q) F.a[q] = Fs[9 * a + q];
            blk HF = blk_mul(Hd, F);
            blk Ha = (a == d) ? Hd : face_block(A.pool, fd[a], m, n, i, j);
            zd s = {0.0, 0.0};
#pragma unroll
            for (int q = 0; q < 9; ++q) s += conj_mul(Ha.a[q], HF.a[q]);
            if (a < d) cross += s;
            else tdd += s;
        }
    }
    double v[2] = {cross.re, tdd.re};
    wg_sum<2>(v, S);
    if (threadIdx.x == 0) {
        double* tp = A.tp + (size_t)(B.tile0 + t) * 8;
        tp[4] = v[0];
        tp[5] = v[1];
    }
}

// low-rank faces: tr(X Y) with X = Ua^H Ud (ka x kd), Y = Vd^H (I (x) F_da) Va (kd x ka)
template <typename T>
__device__ void cross_lr_block(const CompressArgs& A, int b, Red& S, const zd* Fs)
{
    const BlockIn B = A.blocks[b];
    const int m = B.rs, n = B.cs, d = A.d, L = A.L;
    const FaceDesc* fd = A.faces + (size_t)b * L;
    const FaceDesc Fd = fd[d];
    double cross = 0.0, tdd = 0.0;
    if (Fd.kk > 0) {
        const int kd = Fd.kk;
        const cx<T>* Ud = (const cx<T>*)(A.pool + Fd.face_off);
        const cx<T>* Vd = Ud + (size_t)3 * m * kd;
        for (int a = 0; a <= d; ++a) {
            const FaceDesc Fa = fd[a];
            double acc = 0.0;
            if (Fa.kk > 0) {
                const int ka = Fa.kk;
                const cx<T>* Ua = (const cx<T>*)(A.pool + Fa.face_off);
                const cx<T>* Va = Ua + (size_t)3 * m * ka;
                blk F;
#pragma unroll
                for (int q = 0; q < 9; ++q) F.a[q] = Fs[9 * a + q];
                for (int q = threadIdx.x; q < ka * kd; q += WG) {
                    const int s = q / kd, tt = q - s * kd;
                    zd X = {0.0, 0.0}, Y = {0.0, 0.0};
                    for (int r = 0; r < 3 * m; ++r) X += conj_mul(ldz(Ua + (size_t)r * ka + s), ldz(Ud + (size_t)r * kd + tt));
                    for (int j = 0; j < n; ++j) {
                        zd va[3], vd[3];
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            va[c] = ldz(Va + (size_t)(3 * j + c) * ka + s);
                            vd[c] = ldz(Vd + (size_t)(3 * j + c) * kd + tt);
                        }
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            zd fv = F.a[3 * c] * va[0] + F.a[3 * c + 1] * va[1] + F.a[3 * c + 2] * va[2];
                            Y += conj_mul(vd[c], fv);
                        }
                    }
                    acc += (X * Y).re;
                }
            }
            double v[1] = {acc};
            wg_sum<1>(v, S);
            if (a < d) cross += v[0];
            else tdd = v[0];
        }
    }
    if (threadIdx.x == 0) {
        double* tp = A.tp + (size_t)B.tile0 * 8;
        tp[4] = cross;
        tp[5] = tdd;
    }
}

__global__ __launch_bounds__(WG) void k_cross_lr(CompressArgs A)
{
    __shared__ Red S;
    __shared__ zd Fs[MAX_L * 9];
    const int b = A.list[blockIdx.x];
    if (!A.st[b].active || A.st[b].stop) return;
    for (int q = threadIdx.x; q < 9 * (A.d + 1); q += WG) Fs[q] = A.Fda[(size_t)b * A.L * 9 + q];
    __syncthreads();
    if (A.mixed) cross_lr_block<float>(A, b, S, Fs);
    else cross_lr_block<double>(A, b, S, Fs);
}

// ---------------------------------------------------------------- finalize the step

__global__ __launch_bounds__(64) void k_final(CompressArgs A)
{
    int q = blockIdx.x * 64 + threadIdx.x;
    if (q >= A.nlist) return;
    const int b = A.list[q];
    BlockState s = A.st[b];
    if (!s.active || s.stop) return;
    const BlockIn B = A.blocks[b];
    const int d = A.d;
    double cross = 0.0, tdd = 0.0;
    int nt = B.lowrank ? 1 : B.ntile;
    for (int t = 0; t < nt; ++t) {
        const double* tp = A.tp + (size_t)(B.tile0 + t) * 8;
        cross += tp[4];
        tdd += tp[5];
    }
    s.norm2 += 2.0 * cross + tdd;
    const double eps = block_eps(A, B);
    if (!(sqrt(s.hn2 * s.fn2) > eps * sqrt(fmax(s.norm2, 0.0)))) {
        s.rank = d;  // the sub-tolerance pair is dropped
        s.active = 0;
    } else {
        s.rank = d + 1;
        const FaceDesc f = A.faces[(size_t)b * A.L + d];
        if (f.kk > s.aca_max) s.aca_max = f.kk;
        if (s.nextk < 0 || d + 1 == A.L) {
            s.active = 0;
        } else {
            s.k = s.nextk;
            if (!alloc_step(A, b, d + 1, s.k)) s.active = 0;
        }
    }
    A.st[b] = s;
}

// ---------------------------------------------------------------- dense fallback

// storage for frequency kf of every fallback block of the list, with a selector fibre
__global__ __launch_bounds__(64) void k_fallback_alloc(CompressArgs A, int kf)
{
    int q = blockIdx.x * 64 + threadIdx.x;
    if (q >= A.nlist) return;
    const int b = A.list[q];
    const BlockIn B = A.blocks[b];
    long long fb = dense_face_bytes(A, B);
    long long off = pool_alloc(A, fb + (long long)sizeof(zd) * 9 * A.L);
    FaceDesc f;
    f.face_off = off < 0 ? 0 : off;
    f.fib_off = off < 0 ? 0 : off + fb;
    f.kk = off < 0 ? -1 : 0;
    f.k = kf;
    f.sel = 1;
    f.fp32 = (A.mixed && B.far) ? 1 : 0;
    A.faces[(size_t)b * A.L + kf] = f;
    if (off >= 0) {
        zd* fib = (zd*)(A.pool + f.fib_off);
        for (int k = 0; k < A.L; ++k)
            for (int t = 0; t < 9; ++t)
                fib[(size_t)k * 9 + t] = (k == kf && (t == 0 || t == 4 || t == 8)) ? zd{1.0, 0.0} : zd{0.0, 0.0};
    }
    A.st[b].rank = A.L;
}

// face at frequency kf without residual (one workgroup per tile of a fallback block)
__global__ __launch_bounds__(WG) void k_fallback_face(CompressArgs A, int kf)
{
    const int item = A.list[blockIdx.x];
    const int b = item >> 12, t = item & 4095;
    const BlockIn B = A.blocks[b];
    const int m = B.rs, n = B.cs;
    const FaceDesc F = A.faces[(size_t)b * A.L + kf];
    if (F.kk < 0) return;
    const int p = t * TILE + threadIdx.x;
    if (p < m * n) {
        const int i = p / n, j = p - (p / n) * n;
        blk E = entry_of(A, B, i, j, kf);
        size_t ld = 3 * (size_t)n;
        if (F.fp32) {
            zf* H = (zf*)(A.pool + F.face_off);
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) stz(H + (size_t)(3 * i + a) * ld + 3 * j + c, E.a[3 * a + c]);
        } else {
            zd* H = (zd*)(A.pool + F.face_off);
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) H[(size_t)(3 * i + a) * ld + 3 * j + c] = E.a[3 * a + c];
        }
    }
    if (threadIdx.x == 0)
        atomicAdd((unsigned long long*)&A.st[b].entries, (unsigned long long)min(TILE, m * n - t * TILE));
}

}  // namespace

size_t aca_scratch_doubles(int m, int n, int kmax)
{
    return (size_t)2 * (3 * (size_t)m * kmax + 3 * (size_t)n * kmax + 5 * (size_t)kmax * kmax) + kmax +
           (m + kmax + 1) / 2 + 8;
}

#define BEM_LAUNCH(kern, grid, block, ...)                                                     \
    do {                                                                                       \
        if ((grid) > 0) hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, st, __VA_ARGS__); \
        BEM_HIP_TRY(hipGetLastError());                                                        \
    } while (0)

void launch_init(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_init, (A.nblocks + 255) / 256, 256, A); }
void launch_face_dense(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_face_dense, A.nlist, WG, A); }
void launch_aca(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_aca, A.nlist, WG, A); }
void launch_scan_lr(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_scan_lr, A.nlist, WG, A); }
void launch_pivot(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_pivot, (A.nlist + 63) / 64, 64, A); }
void launch_fibre(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_fibre, A.nlist, WG, A); }
void launch_cross_dense(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_cross_dense, A.nlist, WG, A); }
void launch_cross_lr(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_cross_lr, A.nlist, WG, A); }
void launch_final(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_final, (A.nlist + 63) / 64, 64, A); }
void launch_fallback(const CompressArgs& A, int kf, hipStream_t st)
{
    BEM_LAUNCH(k_fallback_alloc, (A.nlist + 63) / 64, 64, A, kf);
}
void launch_fallback_faces(const CompressArgs& A, int kf, hipStream_t st)
{
    BEM_LAUNCH(k_fallback_face, A.nlist, WG, A, kf);
}

}  // namespace bem
