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

// block (i, j) of a stored dense face (row-major 3m x 3n, complex64 or complex128)
__device__ __forceinline__ blk face_block(const char* pool, const FaceDesc& f, int n, int i, int j)
{
    blk b;
    const size_t ld = 3 * (size_t)n;
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

__device__ __forceinline__ blk fibre_at(const char* pool, const FaceDesc& f, int k)
{
    return ld_blk9((const zd*)(pool + f.fib_off) + (size_t)k * 9);
}

// E -= sum_{a<d} H_a[i,j] f_a[k]   (the 3D approximation C^(d-1) at (i, j, k))
__device__ __forceinline__ void sub_residual(blk& E, const CompressArgs& A, const FaceDesc* fd, int d, int n, int i,
                                             int j, int k)
{
    for (int a = 0; a < d; ++a) {
        const FaceDesc f = fd[a];
        if (f.kk < 0 || (f.sel && f.k != k)) continue;
        blk H = face_block(A.pool, f, n, i, j);
        blk fk = fibre_at(A.pool, f, k);
        blk_mul_sub(E, H, fk);
    }
}

// the share of lane u (of a group of lpp) in the residual of E: faces a = u, u + lpp, ...
__device__ __forceinline__ void sub_residual_share(blk& E, const CompressArgs& A, const FaceDesc* fd, int d, int n,
                                                   int i, int j, int k, int u, int lpp)
{
    for (int a = u; a < d; a += lpp) {
        const FaceDesc f = fd[a];
        if (f.kk < 0 || (f.sel && f.k != k)) continue;
        blk H = face_block(A.pool, f, n, i, j);
        blk fk = fibre_at(A.pool, f, k);
        blk_mul_sub(E, H, fk);
    }
}

// lanes per pair for the rule of a pair class: regular 1, near level 1 / 2: 4 / 16 (one
// sub-triangle each), self: a wavefront (angular lines round robin)
__device__ __forceinline__ int pair_lanes(int cls)
{
    return cls == CLS_REGULAR ? 1 : (cls == CLS_NEAR1 ? 4 : (cls == CLS_NEAR2 ? 16 : 64));
}

// sum of E over the aligned groups of lpp lanes (lpp a power of two dividing 64); every
// lane of the wavefront must take part
__device__ __forceinline__ void group_sum(blk& E, int lpp)
{
    for (int o = lpp >> 1; o >= 1; o >>= 1) {
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            E.a[t].re += __shfl_xor(E.a[t].re, o, 64);
            E.a[t].im += __shfl_xor(E.a[t].im, o, 64);
        }
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
    size_t zs = B.f32 ? sizeof(zf) : sizeof(zd);
    return ((long long)zs * 9 * B.rs * B.cs + 15) & ~15LL;
}

// Reserve the storage of step d of block b (dense face + fibre); false on pool overflow.
__device__ bool alloc_step(const CompressArgs& A, int b, int d, int k)
{
    const BlockIn B = A.blocks[b];
    const long long fb = dense_face_bytes(A, B);
    const long long off = pool_alloc(A, fb + (long long)sizeof(zd) * 9 * A.L);
    if (off < 0) return false;
    FaceDesc f;
    f.face_off = off;
    f.fib_off = off + fb;
    f.kk = 0;
    f.k = k;
    f.sel = 0;
    f.fp32 = B.f32;
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
    s.aca_dense = 0;
    s.pad = 0;
    s.aca_cols = 0;
    s.norm2 = 0.0;
    s.hn2 = s.fmax2 = s.s3max = s.fn2 = 0.0;
    s.entries = 0;
    for (int t = 0; t < 9; ++t) s.pinv[t] = {0.0, 0.0};
    for (int k = 0; k < A.L; ++k) A.used[(size_t)b * A.L + k] = 0;
    if (!alloc_step(A, b, 0, 0)) s.active = 0;
    A.st[b] = s;
}

// ---------------------------------------------------------------- dense faces

// Entry of a regular pair for the face kernels: PATH 1 / 2 = FP32 / FP64 regular rule.
// KOP: 0 = V, 1 = K or I/2 + K (the free term sits on i == j, never a regular pair),
// 2 = entry table.
template <int KOP, int PATH>
__device__ __forceinline__ blk pair_entry(const CompressArgs& A, int gi, int gj, int k)
{
    if constexpr (KOP == 2) {
        return entry_dispatch<false>(A.c, OP_TABLE, gi, gj, k);
    } else {
        blk out;
        if constexpr (PATH == 1)
            entry_regular<float>(A.c.geo, KOP, gi, gj, A.c.fr.sf[k], A.c.fr.sinvf[k], A.c.mf, out);
        else
            entry_regular<double>(A.c.geo, KOP, gi, gj, A.c.fr.s[k], A.c.fr.sinv[k], A.c.md, out);
        return out;
    }
}

// E -= sum_{a<d} H_a[i,j] f_a[k] over the dense faces of an iterating block (precision of
// the faces known at compile time).
template <bool F32>
__device__ __forceinline__ void sub_residual_t(blk& E, const char* pool, const FaceDesc* fd, int d, int n, int i,
                                               int j, int k)
{
    const size_t ld = 3 * (size_t)n;
#pragma unroll 2
    for (int a = 0; a < d; ++a) {
        const FaceDesc f = fd[a];
        blk H;
        if constexpr (F32) {
            const zf* Hp = (const zf*)(pool + f.face_off);
#pragma unroll
            for (int x = 0; x < 3; ++x)
#pragma unroll
                for (int c = 0; c < 3; ++c) H.a[3 * x + c] = ldz(Hp + (size_t)(3 * i + x) * ld + 3 * j + c);
        } else {
            const zd* Hp = (const zd*)(pool + f.face_off);
#pragma unroll
            for (int x = 0; x < 3; ++x)
#pragma unroll
                for (int c = 0; c < 3; ++c) H.a[3 * x + c] = Hp[(size_t)(3 * i + x) * ld + 3 * j + c];
        }
        const blk fk = fibre_at(pool, f, k);
        blk_mul_sub(E, H, fk);
    }
}

// pair number p of lane `lane` in tile t of block B, or -1
__device__ __forceinline__ int tile_pair(const CompressArgs& A, const BlockIn& B, int t, int lane)
{
    const int q = t * TILE + lane;
    if (t >= B.ntr || q >= B.nreg) return -1;
    return B.pair0 < 0 ? q : A.pairs[B.pair0 + q];
}

// tile partials: [0] sigma_3 max, [1] pivot pair, [2] sum |H|^2, [3] max block |H|^2,
//                [4] cross re, [5] t_dd re
template <int KOP, int PATH>
__global__ __launch_bounds__(WG) void k_face_dense(CompressArgs A)
{
    constexpr bool F32 = PATH == 1;
    __shared__ Red S;
    const int item = A.list[blockIdx.x];
    const int b = item >> 12, t = item & 4095;
    if (!A.st[b].active) return;
    const BlockIn B = A.blocks[b];
    const int m = B.rs, n = B.cs, d = A.d;
    const int k = A.st[b].k;
    const FaceDesc* fd = A.faces + (size_t)b * A.L;
    const FaceDesc F = fd[d];
    const int p = tile_pair(A, B, t, threadIdx.x);
    double s3 = -1.0, e2 = 0.0;
    int pi = 0x7fffffff;
    if (p >= 0) {
        const int i = p / n, j = p - (p / n) * n;
        blk E = pair_entry<KOP, PATH>(A, B.rb + i, B.cb + j, k);
        sub_residual_t<F32>(E, A.pool, fd, d, n, i, j, k);
        const size_t ld = 3 * (size_t)n;
        if constexpr (F32) {
            zf* H = (zf*)(A.pool + F.face_off);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const zd v = E.a[3 * a + c];
                    const zf w = {(float)v.re, (float)v.im};
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
        atomicAdd((unsigned long long*)&A.st[b].entries, (unsigned long long)max(0, min(TILE, B.nreg - t * TILE)));
    }
}

// Face kernel for the tiles of near and self pairs (tile t >= ntr of a block): tiles of one
// class, a group of pair_lanes(cls) lanes per pair, each lane one or more units of the rule
// and a share of the residual, summed over the group.  F32: faces stored in complex64.
template <int KOP, bool F32, bool SELF>
__global__ __launch_bounds__(WG) void k_face_general(CompressArgs A)
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
    int tl = t - B.ntr, cls, base, cnt;
    const int t1 = (B.n1 + WG / 4 - 1) / (WG / 4), t2 = (B.n2 + WG / 16 - 1) / (WG / 16);
    if (SELF) {
        cls = CLS_SELF;
        tl -= t1 + t2;
        base = B.nreg + B.n1 + B.n2;
        cnt = B.n3;
    } else if (tl < t1) {
        cls = CLS_NEAR1;
        base = B.nreg;
        cnt = B.n1;
    } else {
        cls = CLS_NEAR2;
        tl -= t1;
        base = B.nreg + B.n1;
        cnt = B.n2;
    }
    const int lpp = pair_lanes(cls), ppt = WG / lpp;
    const int q = tl * ppt + (int)threadIdx.x / lpp, u = threadIdx.x % lpp;
    const bool valid = q < cnt;
    const int p = valid ? A.pairs[B.pair0 + base + q] : 0;
    const int i = p / n, j = p - (p / n) * n;
    blk E = blk_zero();
    if (valid) {
        const int nu = rule_units(cls, A.c.qt);
        for (int uu = u; uu < nu; uu += lpp) {
            blk e;
            if constexpr (SELF)
                self_unit<KOP>(A.c.geo, B.cb + j, uu, A.c.fr.s[k], A.c.fr.sinv[k], A.c.md, A.c.qt, e);
            else
                near_unit<KOP>(A.c.geo, B.rb + i, B.cb + j, cls, uu, A.c.fr.s[k], A.c.fr.sinv[k], A.c.md, A.c.qt, e);
#pragma unroll
            for (int x = 0; x < 9; ++x) E.a[x] += e.a[x];
        }
        if (u == 0 && A.op == OP_HK && B.rb + i == B.cb + j) {
            E.a[0].re += 0.5;
            E.a[4].re += 0.5;
            E.a[8].re += 0.5;
        }
        sub_residual_share(E, A, fd, d, n, i, j, k, u, lpp);
    }
    group_sum(E, lpp);
    double s3 = -1.0, e2 = 0.0;
    int pi = 0x7fffffff;
    if (valid && u == 0) {
        const size_t ld = 3 * (size_t)n;
        if constexpr (F32) {
            zf* H = (zf*)(A.pool + F.face_off);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const zd v = E.a[3 * a + c];
                    const zf w = {(float)v.re, (float)v.im};
                    H[(size_t)(3 * i + a) * ld + 3 * j + c] = w;
                    E.a[3 * a + c] = {(double)w.re, (double)w.im};
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
        atomicAdd((unsigned long long*)&A.st[b].entries, (unsigned long long)max(0, min(ppt, cnt - tl * ppt)));
    }
    (void)m;
}

__global__ __launch_bounds__(WG) void k_classify(DevCtx c, const BlockIn* blocks, const int* list,
                                                 const long long* off, unsigned char* cls)
{
    const BlockIn B = blocks[list[blockIdx.x]];
    unsigned char* o = cls + off[blockIdx.x];
    for (int p = threadIdx.x; p < B.rs * B.cs; p += WG) {
        const int i = p / B.cs, j = p - i * B.cs;
        o[p] = (unsigned char)pair_class(c.geo, B.rb + i, B.cb + j, c.qt);
    }
}

// ---------------------------------------------------------------- per-slice ACA of far faces

// Scratch of one face: ACA columns and the small matrices of the recompression.
struct AcaWork {
    zd *U, *V;        // 3m x kmax, 3n x kmax column-major
    zd *G, *RU, *RV;  // kmax x kmax
    zd *M, *VJ;       // kmax x kmax
    double* dn;       // kmax
    int* usedrow;     // m
    int* order;       // kmax
    int* info;        // [0]: ACA columns of the face in this slot (-1: not resolved)
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
    w.info = w.order + kmax;
    return w;
}

struct AcaShared {
    Red r;
    zd pinv[9];
    double s;
    int piv, flag;
};

// block (i, j) of the stored face H (3m x 3n row-major) minus the cross approximation U V^H
template <typename T>
__device__ __forceinline__ blk aca_residual(const cx<T>* H, int m, int n, const AcaWork& w, int kc, int i, int j)
{
    blk E;
    const size_t ld = 3 * (size_t)n;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) E.a[3 * a + c] = ldz(H + (size_t)(3 * i + a) * ld + 3 * j + c);
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

// Matrix-valued partial-pivot ACA of the stored face with rank-3 steps and sigma_3 pivots
// (the matrix form of the pivoting of Algorithm 1).  Stops once the newest 3 columns satisfy
// ||U_k||_F ||V_k||_F <= tol, or when a residual row without a regular block is itself
// below tol.  Returns the number of columns, or -1 when the face is not resolved within cap
// columns short of 3 min(m, n) (or MAX_FAIL rows in a row have no regular pivot, or a row skipped that way is
// left at the end): the caller keeps the face dense.
template <typename T>
__device__ int face_aca(const cx<T>* H, int m, int n, const AcaWork& w, int cap, double tol, double amax,
                        AcaShared& S)
{
    for (int i = threadIdx.x; i < m; i += WG) w.usedrow[i] = 0;
    __syncthreads();
    int kc = 0, fails = 0, skipped = 0, irow = 0;
    for (;;) {
        if (kc + 3 > cap) return kc >= 3 * min(m, n) ? kc : -1;  // all of min(m, n) interpolated: exact
        // residual row block irow -> V columns kc..kc+2 (row^H)
        double best = -1.0, rn2 = 0.0;
        int bj = 0x7fffffff;
        for (int j = threadIdx.x; j < n; j += WG) {
            blk E = aca_residual(H, m, n, w, kc, irow, j);
#pragma unroll
            for (int y = 0; y < 3; ++y)
#pragma unroll
                for (int x = 0; x < 3; ++x) w.V[(size_t)(kc + y) * 3 * n + 3 * j + x] = conj(E.a[3 * y + x]);
            rn2 += blk_fro2(E);
            double s3 = blk_sigma3(E);
            if (s3 > best || (s3 == best && j < bj)) {
                best = s3;
                bj = j;
            }
        }
        if (threadIdx.x == 0) w.usedrow[irow] = 1;
        double v1[1] = {rn2};
        wg_sum<1>(v1, S.r);
        rn2 = v1[0];
        wg_argmax(best, bj, S.r);
        if (!(best > PIVOT_RTOL * amax)) {
            if (sqrt(rn2) <= tol) return kc;  // negligible residual row
            ++skipped;
            if (++fails >= MAX_FAIL) return -1;
            int cand = 0x7fffffff;
            for (int i = threadIdx.x; i < m; i += WG)
                if (!w.usedrow[i] && i < cand) cand = i;
            double cv = cand == 0x7fffffff ? -1.0 : 1.0;
            wg_argmax(cv, cand, S.r);
            if (cv < 0.0) return -1;  // every row visited, a skipped row remains
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
        // residual column block bj -> U columns kc..kc+2 = column * P^{-1}
        double best2 = -1.0, un2 = 0.0;
        int bi2 = 0x7fffffff;
        for (int i = threadIdx.x; i < m; i += WG) {
            blk E = aca_residual(H, m, n, w, kc, i, bj);
            blk Pi;
#pragma unroll
            for (int t = 0; t < 9; ++t) Pi.a[t] = S.pinv[t];
            blk Un = blk_mul(E, Pi);
#pragma unroll
            for (int y = 0; y < 3; ++y)
#pragma unroll
                for (int x = 0; x < 3; ++x) w.U[(size_t)(kc + x) * 3 * m + 3 * i + y] = Un.a[3 * y + x];
            un2 += blk_fro2(Un);
            double s3 = w.usedrow[i] ? -1.0 : blk_sigma3(Un);
            if (s3 > best2 || (s3 == best2 && i < bi2)) {
                best2 = s3;
                bi2 = i;
            }
        }
        double v2[1] = {un2};
        wg_sum<1>(v2, S.r);
        kc += 3;
        if (sqrt(v2[0] * rn2) <= tol) return kc;
        wg_argmax(best2, bi2, S.r);
        if (best2 < 0.0) return skipped ? -1 : kc;  // every row is a pivot row: exact
        irow = bi2;
    }
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

// Recompression (eq. (ACA)) of U (3m x kc), V (3n x kc): QR of both, SVD of R_U R_V^H,
// truncation to the smallest kk with sqrt(sum_{t >= kk} s_t^2) <= tol.  When the
// factors Ubar = Q_U Uc Sigma (3m x kk) and Vbar = Q_V Vc (3n x kk) take less memory than
// the dense face, they are written row-major over the face storage Hout (precision T)
// and kk is returned; otherwise 0 (the face stays dense).
template <typename T>
__device__ int face_recompress(cx<T>* Hout, int m, int n, const AcaWork& w, int kc, double tol, AcaShared& S)
{
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
            if (sqrt(tail + s * s) <= tol) {
                tail += s * s;
                --kk;
            } else {
                break;
            }
        }
        if (tot > 0.0 && kk == 0) kk = 1;
        if ((long long)kk * (m + n) >= 3LL * m * n) kk = 0;  // no saving over the dense face
        S.piv = kk;
    }
    __syncthreads();
    const int kk = S.piv;
    if (kk <= 0) return 0;
    cx<T>* Ub = Hout;
    cx<T>* Vb = Hout + (size_t)3 * m * kk;
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

// ---------------------------------------------------------------- recompression in LDS

// Faces with kc <= KF columns recompress with their kc x kc matrices in LDS (one workgroup
// per face, kc^2 complex128 = 144 KiB at kc = 96); larger ones take the global-memory path.
constexpr int KF = 96;
constexpr int GCH = 4;  // rows of a Gram chunk staged in LDS

struct RecompShared {
    zd m[KF * KF];       // kc x kc column-major working matrix
    zd stage[GCH * KF];  // Gram row chunk
    zd tau[KF];          // reflector coefficients of the pivoted QR
    double sv[KF];       // column norms / singular values
    int order[KF];
    int perm[KF];        // column order of the pivoted QR
};

// Lm (kc x kc, column-major, full Hermitian) = X^H X for X (rows x kc, column-major, global).
// 4 x 4 output tiles per thread over the upper tile triangle; X streamed through LDS.
__device__ void lds_gram(const zd* X, int rows, int kc, zd* Lm, zd* stage)
{
    const int nt = (kc + 3) >> 2, ntri = nt * (nt + 1) / 2;
    for (int base = 0; base < ntri; base += WG) {
        const int tt = base + threadIdx.x;
        const bool act = tt < ntri;
        int tj = 0, ti = 0;
        if (act) {
            tj = (int)((sqrt(8.0 * tt + 1.0) - 1.0) * 0.5);
            while ((tj + 1) * (tj + 2) / 2 <= tt) ++tj;
            while (tj * (tj + 1) / 2 > tt) --tj;
            ti = tt - tj * (tj + 1) / 2;
        }
        zd acc[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = {0.0, 0.0};
        for (int r0 = 0; r0 < rows; r0 += GCH) {
            const int nr = min(GCH, rows - r0);
            __syncthreads();
            for (int q = threadIdx.x; q < GCH * kc; q += WG) {
                const int c = q / GCH, r = q - c * GCH;
                stage[r * kc + c] = r < nr ? X[(size_t)c * rows + r0 + r] : zd{0.0, 0.0};
            }
            __syncthreads();
            if (act) {
                for (int r = 0; r < nr; ++r) {
                    zd a[4], b[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int ca = 4 * ti + u, cb = 4 * tj + u;
                        a[u] = ca < kc ? stage[r * kc + ca] : zd{0.0, 0.0};
                        b[u] = cb < kc ? stage[r * kc + cb] : zd{0.0, 0.0};
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[u][v] += conj_mul(a[u], b[v]);
                }
            }
        }
        if (act) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = 4 * ti + u, j = 4 * tj + v;
                    if (i < kc && j < kc && i <= j) {
                        Lm[(size_t)j * kc + i] = acc[u][v];
                        Lm[(size_t)i * kc + j] = conj(acc[u][v]);
                    }
                }
        }
    }
    __syncthreads();
}

// Cholesky in place: Lm = R^H R with R upper (stored in the upper triangle, lower zeroed);
// a pivot without positive mass gives a zero row.  Returns the smallest pivot (before the
// square root) to every thread.
__device__ double lds_cholesky(zd* Lm, int kc, AcaShared& S)
{
    double pmin = 1e300;
    for (int k = 0; k < kc; ++k) {
        if (threadIdx.x == 0) {
            const double p = Lm[(size_t)k * kc + k].re;
            pmin = fmin(pmin, p);
            S.s = p > 1e-24 ? sqrt(p) : 0.0;
        }
        __syncthreads();
        const double rkk = S.s;
        for (int j = k + threadIdx.x; j < kc; j += WG) {
            const zd g = Lm[(size_t)j * kc + k];
            Lm[(size_t)j * kc + k] = (j == k) ? zd{rkk, 0.0} : (rkk > 0.0 ? g * (1.0 / rkk) : zd{0.0, 0.0});
        }
        __syncthreads();
        const int rem = kc - k - 1;
        for (int q = threadIdx.x; q < rem * rem; q += WG) {
            const int jj = k + 1 + q / rem, ii = k + 1 + q % rem;
            if (ii <= jj) Lm[(size_t)jj * kc + ii] -= conj_mul(Lm[(size_t)ii * kc + k], Lm[(size_t)jj * kc + k]);
        }
        __syncthreads();
    }
    for (int q = threadIdx.x; q < kc * kc; q += WG)
        if (q % kc > q / kc) Lm[q] = {0.0, 0.0};
    if (threadIdx.x == 0) S.s = pmin;
    __syncthreads();
    pmin = S.s;
    __syncthreads();
    return pmin;
}

// X (rows x kc, column-major, global) <- X R^{-1}, R upper in Lm; blocks of 8 columns per
// pass, one row per thread; zero pivots give zero columns.
__device__ void lds_trsm(zd* X, int rows, const zd* Lm, int kc)
{
    constexpr int NB = 8;
    for (int r = threadIdx.x; r < rows; r += WG) {
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

// The pivoted QR of the core matrix stops once its remaining columns are below
// QRCP_FRAC tol; the SVD truncation of the kept rows then has sqrt(1 - QRCP_FRAC^2) of the
// tolerance left.
constexpr double QRCP_FRAC = 0.25;

// Smallest Cholesky pivot of the column-scaled Gram (unit diagonal) that a single CholeskyQR
// accepts: below it (cond above ~1e5) the factor is refined by a second pass.
constexpr double CQ2_PIVOT = 1e-10;

// Column scaling + CholeskyQR of X (rows x kc), repeated once (CholeskyQR2) when the first
// pass meets a pivot below CQ2_PIVOT.  On return Q = X T^{-1} with T upper in Tout (X holds
// X D^{-1}, or Q1 = X D^{-1} R1^{-1} after two passes) and R = R_fact D in Rout, R_fact the
// triangular factor of X D^{-1}; both kc x kc column-major in global scratch.
__device__ void lds_qr(zd* X, int rows, int kc, zd* Rout, zd* Tout, zd* Lm, RecompShared& L, AcaShared& S)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int c = wv; c < kc; c += WG / 64) {
        double s = 0.0;
        for (int r = lane; r < rows; r += 64) s += abs2(X[(size_t)c * rows + r]);
        s = wsum(s);
        if (lane == 0) L.sv[c] = sqrt(s);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < rows * kc; q += WG) {
        const double dc = L.sv[q / rows];
        X[q] = dc > 0.0 ? X[q] * (1.0 / dc) : zd{0.0, 0.0};
    }
    __syncthreads();
    lds_gram(X, rows, kc, Lm, L.stage);
    const double pmin = lds_cholesky(Lm, kc, S);
    if (pmin >= CQ2_PIVOT) {
        for (int q = threadIdx.x; q < kc * kc; q += WG) {
            Tout[q] = Lm[q];
            Rout[q] = Lm[q] * L.sv[q / kc];
        }
        __syncthreads();
        return;
    }
    lds_trsm(X, rows, Lm, kc);
    for (int q = threadIdx.x; q < kc * kc; q += WG) Tout[q] = Lm[q];  // R1 (temporarily)
    __syncthreads();
    lds_gram(X, rows, kc, Lm, L.stage);
    lds_cholesky(Lm, kc, S);
    // Rout = R2 R1 D, then Tout = R2
    for (int q = threadIdx.x; q < kc * kc; q += WG) {
        const int i = q % kc, j = q / kc;
        zd s = {0.0, 0.0};
        for (int t = i; t <= j; ++t) s += Lm[(size_t)t * kc + i] * Tout[(size_t)j * kc + t];
        Rout[q] = i <= j ? s * L.sv[j] : zd{0.0, 0.0};
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kc * kc; q += WG) Tout[q] = Lm[q];
    __syncthreads();
}

// Householder QR with column pivoting of A = Lm (kc x kc, column-major) in place (complex
// reflectors H = I - tau v v^H, v[0] = 1, v below the diagonal), stopped at the first step
// whose remaining columns have Frobenius norm <= delta.  Returns the number of steps k;
// tau in L.tau, the column order in L.perm, the remaining squared norm in *rest2.
__device__ int lds_qrcp(zd* Lm, int kc, double delta, RecompShared& L, AcaShared& S, double* rest2)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int c = wv; c < kc; c += WG / 64) {
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
        // remaining norm and pivot column (wavefront 0)
        if (wv == 0) {
            double t = 0.0, best = -1.0;
            int bi = 0x7fffffff;
            for (int c = j + lane; c < kc; c += 64) {
                t += L.sv[c];
                if (L.sv[c] > best || (L.sv[c] == best && c < bi)) {
                    best = L.sv[c];
                    bi = c;
                }
            }
            t = wsum(t);
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                const double ob = __shfl_xor(best, o, 64);
                const int oi = __shfl_xor(bi, o, 64);
                if (ob > best || (ob == best && oi < bi)) {
                    best = ob;
                    bi = oi;
                }
            }
            if (lane == 0) {
                S.s = t;
                S.piv = bi;
            }
        }
        __syncthreads();
        const double rest = S.s;
        const int p = S.piv;
        if (sqrt(fmax(rest, 0.0)) <= delta) break;
        if (p != j) {
            for (int r = threadIdx.x; r < kc; r += WG) {
                const zd a = Lm[(size_t)j * kc + r];
                Lm[(size_t)j * kc + r] = Lm[(size_t)p * kc + r];
                Lm[(size_t)p * kc + r] = a;
            }
            if (threadIdx.x == 0) {
                const double sv = L.sv[j];
                L.sv[j] = L.sv[p];
                L.sv[p] = sv;
                const int pm = L.perm[j];
                L.perm[j] = L.perm[p];
                L.perm[p] = pm;
            }
        }
        __syncthreads();
        // reflector of column j (wavefront 0): beta = -sign(Re alpha) ||x||
        zd* aj = Lm + (size_t)j * kc;
        if (wv == 0) {
            double x2 = 0.0;
            for (int r = j + 1 + lane; r < kc; r += 64) x2 += abs2(aj[r]);
            x2 = wsum(x2);
            if (lane == 0) {
                const zd al = aj[j];
                zd tau = {0.0, 0.0}, sc = {0.0, 0.0};
                if (x2 > 0.0 || al.im != 0.0) {
                    const double nrm = sqrt(abs2(al) + x2);
                    const double beta = al.re >= 0.0 ? -nrm : nrm;
                    tau = {(beta - al.re) / beta, -al.im / beta};
                    sc = zdiv(zd{1.0, 0.0}, al - zd{beta, 0.0});
                    aj[j] = {beta, 0.0};
                }
                L.tau[j] = tau;
                S.pinv[0] = sc;
            }
        }
        __syncthreads();
        const zd sc = S.pinv[0];
        for (int r = j + 1 + threadIdx.x; r < kc; r += WG) aj[r] = aj[r] * sc;
        __syncthreads();
        // apply H^H to the columns j + 1 .. kc - 1 (one wavefront per column), refresh norms
        const zd tc = conj(L.tau[j]);
        for (int c = j + 1 + wv; c < kc; c += WG / 64) {
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
            const zd wv2 = tc * zd{wr, wi};
            double s = 0.0;
            for (int r = j + lane; r < kc; r += 64) {
                const zd v = r == j ? zd{1.0, 0.0} : aj[r];
                const zd a = ac[r] - v * wv2;
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

// One-sided Jacobi on the ncol columns (length rows, stride ld) at Lm: Lm <- B VJ with
// orthogonal columns, rotations not accumulated.  JGL lanes of a wavefront per column pair.
constexpr int JGL = 8;
__device__ void lds_jacobi(zd* Lm, int rows, int ncol, int ld, AcaShared& S)
{
    const int np = ncol + (ncol & 1);
    const int g = threadIdx.x / JGL, gl = threadIdx.x % JGL;
    if (ncol < 2) return;
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (threadIdx.x == 0) S.flag = 0;
        __syncthreads();
        for (int rnd = 0; rnd < np - 1; ++rnd) {
            for (int pr = g; pr < np / 2; pr += WG / JGL) {
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
                double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
                for (int r = gl; r < rows; r += JGL) {
                    const zd a = mp[r], b = mq[r];
                    al += abs2(a);
                    be += abs2(b);
                    const zd c = conj_mul(a, b);
                    gr += c.re;
                    gi += c.im;
                }
#pragma unroll
                for (int o = 1; o < JGL; o <<= 1) {
                    al += __shfl_xor(al, o, 64);
                    be += __shfl_xor(be, o, 64);
                    gr += __shfl_xor(gr, o, 64);
                    gi += __shfl_xor(gi, o, 64);
                }
                const double gabs = sqrt(gr * gr + gi * gi);
                if (!(gabs > 1e-12 * sqrt(al * be)) || gabs == 0.0) continue;
                if (gl == 0) S.flag = 1;
                const zd e = {gr / gabs, gi / gabs};
                const double zeta = (be - al) / (2.0 * gabs);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                const zd ce = conj(e);
                for (int r = gl; r < rows; r += JGL) {
                    const zd a = mp[r], b = mq[r] * ce;
                    mp[r] = c * a - s * b;
                    mq[r] = (s * a + c * b) * e;
                }
            }
            __syncthreads();
        }
        const int f = S.flag;
        __syncthreads();
        if (!f) break;
    }
}

// Y <- R^{-1} Y in place for kk columns (column s at Y + s * ldy, kc rows; LDS or global),
// R upper (kc x kc, column-major, global): right-looking, all threads per step.
__device__ void backsub_cols(const zd* R, int kc, zd* Y, int ldy, int kk)
{
    for (int i = kc - 1; i >= 0; --i) {
        const double d = R[(size_t)i * kc + i].re;
        for (int s = threadIdx.x; s < kk; s += WG) {
            const zd v = Y[(size_t)s * ldy + i];
            Y[(size_t)s * ldy + i] = d > 0.0 ? v * (1.0 / d) : zd{0.0, 0.0};
        }
        __syncthreads();
        for (int q = threadIdx.x; q < i * kk; q += WG) {
            const int t = q % i, s = q / i;
            Y[(size_t)s * ldy + t] -= R[(size_t)i * kc + t] * Y[(size_t)s * ldy + i];
        }
        __syncthreads();
    }
}

// out (rows x kk, row-major, precision T) = X (rows x kc, column-major, global) Y (kc x kk,
// column-major in LDS); one row per thread, 16 columns per pass.
template <typename T>
__device__ void out_gemm(cx<T>* out, const zd* X, int rows, int kc, const zd* Y, int kk)
{
    constexpr int CH = 16;
    for (int r = threadIdx.x; r < rows; r += WG) {
        for (int s0 = 0; s0 < kk; s0 += CH) {
            zd acc[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) acc[u] = {0.0, 0.0};
            for (int t = 0; t < kc; ++t) {
                const zd x = X[(size_t)t * rows + r];
#pragma unroll
                for (int u = 0; u < CH; ++u)
                    if (s0 + u < kk) acc[u] += x * Y[(size_t)(s0 + u) * kc + t];
            }
#pragma unroll
            for (int u = 0; u < CH; ++u)
                if (s0 + u < kk) stz(out + (size_t)r * kk + s0 + u, acc[u]);
        }
    }
    __syncthreads();
}

// Recompression (eq. (ACA)) of U (3m x kc), V (3n x kc), kc <= KF, in LDS:
//   U = Q_U R_U, V = Q_V R_V (CholeskyQR, column-scaled), M = R_U R_V^H,
//   M P = Q_M R (Householder QR with column pivoting, stopped when the remaining columns
//   are below QRCP_FRAC tol: M ~ Q_M B with B = R_top P^T, k' rows),
//   B^H VJ = W (one-sided Jacobi, W with orthogonal columns sigma_s), VJ_s = B W_s / sigma_s^2,
//   so M ~ sum_s (Q_M VJ_s) sigma_s (W_s / sigma_s)^H, truncated at tol (the dropped QR part
//   counted in the tail); Ubar_s = Q_U Q_M VJ_s sigma_s, Vbar_s = Q_V W_s / sigma_s.
// Factors are written row-major over the face storage Hout when they take less memory than
// the dense face (returns kk), else 0.  Scratch: G = T_U, VJ = T_V, RU = R_U then B^H then
// Vbar coefficients, RV = R_V then Ubar coefficients, M = the pivoted QR.
template <typename T>
__device__ int face_recompress_lds(cx<T>* Hout, int m, int n, const AcaWork& w, int kc, double tol,
                                   RecompShared& L, AcaShared& S)
{
    zd* Lm = L.m;
    lds_qr(w.U, 3 * m, kc, w.RU, w.G, Lm, L, S);
    lds_qr(w.V, 3 * n, kc, w.RV, w.VJ, Lm, L, S);
    for (int q = threadIdx.x; q < kc * kc; q += WG) {
        const int i = q % kc, j = q / kc;
        zd s = {0.0, 0.0};
        for (int t = max(i, j); t < kc; ++t) s += mul_conj(w.RU[(size_t)t * kc + i], w.RV[(size_t)t * kc + j]);
        Lm[q] = s;
    }
    __syncthreads();
    double rest2 = 0.0;
    const int kq = lds_qrcp(Lm, kc, QRCP_FRAC * tol, L, S, &rest2);
    if (kq == 0) return 0;
    // keep the pivoted QR, form B^H (kc x kq): B^H[perm[c]][i] = conj(R[i][c]), i <= c
    for (int q = threadIdx.x; q < kc * kc; q += WG) w.M[q] = Lm[q];
    __syncthreads();
    for (int q = threadIdx.x; q < kc * kq; q += WG) {
        const int c = q % kc, i = q / kc;
        const zd v = i <= c ? conj(w.M[(size_t)c * kc + i]) : zd{0.0, 0.0};
        Lm[(size_t)i * kc + L.perm[c]] = v;
        w.RU[(size_t)i * kc + L.perm[c]] = v;
    }
    __syncthreads();
    lds_jacobi(Lm, kc, kq, kc, S);
    for (int c = threadIdx.x; c < kq; c += WG) {
        double s = 0.0;
        for (int r = 0; r < kc; ++r) s += abs2(Lm[(size_t)c * kc + r]);
        L.sv[c] = sqrt(s);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < kq; c += WG) {
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
        S.piv = kk;
    }
    __syncthreads();
    const int kk = S.piv;
    if (kk <= 0) return 0;
    // Ubar coefficients -> RV: sigma_s Q_M [VJ_s; 0], VJ_s = B W_s / sigma_s^2 (kq entries)
    for (int q = threadIdx.x; q < kc * kk; q += WG) {
        const int i = q % kc, s = q / kc;
        zd v = {0.0, 0.0};
        if (i < kq) {
            const int c = L.order[s];
            const double sg = L.sv[c];
            for (int r = 0; r < kc; ++r) v += conj_mul(w.RU[(size_t)i * kc + r], Lm[(size_t)c * kc + r]);
            v = sg > 0.0 ? v * (1.0 / sg) : zd{0.0, 0.0};
        }
        w.RV[(size_t)s * kc + i] = v;
    }
    __syncthreads();
    // Vbar coefficients -> RU: W_s / sigma_s
    for (int q = threadIdx.x; q < kc * kk; q += WG) {
        const int r = q % kc, s = q / kc;
        const int c = L.order[s];
        const double sg = L.sv[c];
        w.RU[(size_t)s * kc + r] = sg > 0.0 ? Lm[(size_t)c * kc + r] * (1.0 / sg) : zd{0.0, 0.0};
    }
    __syncthreads();
    cx<T>* Ub = Hout;
    cx<T>* Vb = Hout + (size_t)3 * m * kk;
    for (int q = threadIdx.x; q < kc * kk; q += WG) Lm[q] = w.RV[q];
    __syncthreads();
    // apply Q_M = H_0 ... H_{kq-1} (H = I - tau v v^H) to the Ubar coefficients, one
    // wavefront per column
    {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        for (int jq = kq - 1; jq >= 0; --jq) {
            const zd tj = L.tau[jq];
            const zd* vj = w.M + (size_t)jq * kc;
            for (int s = wv; s < kk; s += WG / 64) {
                zd* y = Lm + (size_t)s * kc;
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
    }
    backsub_cols(w.G, kc, Lm, kc, kk);
    out_gemm(Ub, w.U, 3 * m, kc, Lm, kk);
    for (int q = threadIdx.x; q < kc * kk; q += WG) Lm[q] = w.RU[q];
    __syncthreads();
    backsub_cols(w.VJ, kc, Lm, kc, kk);
    out_gemm(Vb, w.V, 3 * n, kc, Lm, kk);
    return kk;
}

// ACA stage of one stored dense face: ||H||_F, the pivot scale max |H|, then face_aca;
// returns the column count (-1: not resolved, or a zero face).
template <typename T>
__device__ int face_aca_stage(const cx<T>* H, int m, int n, const AcaWork& w, int cap, double tol, AcaShared& S)
{
    double s2 = 0.0, amax = 0.0;
    const size_t cnt = (size_t)9 * m * n;
    for (size_t q = threadIdx.x; q < cnt; q += WG) {
        const double a2 = abs2(ldz(H + q));
        s2 += a2;
        amax = fmax(amax, a2);
    }
    double v1[1] = {s2};
    wg_sum<1>(v1, S.r);
    amax = sqrt(wg_max(amax, S.r));
    return v1[0] > 0.0 ? face_aca(H, m, n, w, cap, tol, amax, S) : -1;
}

// Recompression stage: kk > 0 (factors written over the face) or 0 (kept dense).
template <typename T>
__device__ int face_recompress_stage(cx<T>* H, int m, int n, const AcaWork& w, int kc, double tol, RecompShared& L,
                                     AcaShared& S)
{
    if (kc <= 0) return 0;
    if (kc <= KF) return face_recompress_lds(H, m, n, w, kc, tol, L, S);
    return face_recompress(H, m, n, w, kc, tol, S);
}

// Absolute tolerance of face d of block b: eps_aca ||C^(r)||_F / ||f_d||_F, so that each
// face-fibre term errs by at most about eps_aca ||C^(r)||_F.
__device__ double face_tol(const CompressArgs& A, int b, const FaceDesc& f, AcaShared& S)
{
    double fn2 = 0.0;
    const zd* fib = (const zd*)(A.pool + f.fib_off);
    for (int q = threadIdx.x; q < 9 * A.L; q += WG) fn2 += abs2(fib[q]);
    double v1[1] = {fn2};
    wg_sum<1>(v1, S.r);
    return v1[0] > 0.0 ? A.eps_aca_far * sqrt(fmax(A.st[b].norm2, 0.0) / v1[0]) : 0.0;
}

// Per-slice ACA pass, one workgroup per listed face (items (block << 8) | d, scratch slot =
// position in the list): k_face_aca leaves the ACA columns in the slot, k_face_recomp
// recompresses them and rewrites the face descriptor.
__global__ __launch_bounds__(WG) void k_face_aca(CompressArgs A)
{
    __shared__ AcaShared S;
    const int item = A.list[blockIdx.x];
    const int b = item >> 8, d = item & 255;
    const BlockIn B = A.blocks[b];
    const FaceDesc f = A.faces[(size_t)b * A.L + d];
    const int m = B.rs, n = B.cs;
    AcaWork w = aca_work(A.scratch + (size_t)blockIdx.x * A.scratch_per_slot, m, n, A.kmax);
    int kc = -1;
    if (f.kk == 0 && !f.sel) {
        const int cap = min(A.kmax, face_aca_cap(m, n));
        const double tol = face_tol(A, b, f, S);
        kc = f.fp32 ? face_aca_stage((const cx<float>*)(A.pool + f.face_off), m, n, w, cap, tol, S)
                    : face_aca_stage((const cx<double>*)(A.pool + f.face_off), m, n, w, cap, tol, S);
    }
    if (threadIdx.x == 0) w.info[0] = kc;
}

__global__ __launch_bounds__(WG) void k_face_recomp(CompressArgs A)
{
    __shared__ AcaShared S;
    __shared__ RecompShared L;
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
    if (kc > 0) {
        const double tol = face_tol(A, b, f, S);
        kk = f.fp32 ? face_recompress_stage((cx<float>*)(A.pool + f.face_off), m, n, w, kc, tol, L, S)
                    : face_recompress_stage((cx<double>*)(A.pool + f.face_off), m, n, w, kc, tol, L, S);
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
        blk P = face_block(A.pool, A.faces[(size_t)b * A.L + d], n, pi / n, pi - (pi / n) * n);
        blk Pi = blk_inv(P);
        for (int t = 0; t < 9; ++t) s.pinv[t] = Pi.a[t];
        A.used[(size_t)b * A.L + s.k] = 1;
    }
    A.st[b] = s;
}

// ---------------------------------------------------------------- fibres

// GEN: blocks whose pivot pair takes the near or self rule (else the regular rule)
template <bool GEN>
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
    {
        const bool gen = A.op != OP_TABLE && pair_class(A.c.geo, B.rb + pi, B.cb + pj, A.c.qt) != CLS_REGULAR;
        if (gen != GEN) return;
    }
    if (threadIdx.x < 9) Pi_s[threadIdx.x] = A.st[b].pinv[threadIdx.x];
    __syncthreads();
    zd* f = (zd*)(A.pool + fd[d].fib_off);
    double fn2 = 0.0, best = -1.0;
    int bk = 0x7fffffff;
    // a near or self pivot pair spreads each entry's rule over a group of lanes
    const int gi = B.rb + pi, gj = B.cb + pj;
    const int cls = GEN ? pair_class(A.c.geo, gi, gj, A.c.qt) : CLS_REGULAR;
    const int lpp = pair_lanes(cls), nu = GEN ? rule_units(cls, A.c.qt) : 1;
    const int u = threadIdx.x % lpp;
    for (int k0 = 0; k0 < L; k0 += WG / lpp) {
        const int k = k0 + threadIdx.x / lpp;
        blk E = blk_zero();
        if (k < L) {
            if constexpr (!GEN) {
                if (A.op == OP_TABLE) E = entry_dispatch<false>(A.c, OP_TABLE, gi, gj, k);
                else if (B.f32)
                    entry_regular<float>(A.c.geo, A.op == OP_V ? 0 : 1, gi, gj, A.c.fr.sf[k], A.c.fr.sinvf[k], A.c.mf, E);
                else
                    entry_regular<double>(A.c.geo, A.op == OP_V ? 0 : 1, gi, gj, A.c.fr.s[k], A.c.fr.sinv[k], A.c.md, E);
            } else {
                for (int uu = u; uu < nu; uu += lpp) {
                    blk e;
                    if (A.op == OP_V) entry_unit<0>(A.c.geo, gi, gj, cls, uu, A.c.fr.s[k], A.c.fr.sinv[k], A.c.md, A.c.qt, e);
                    else entry_unit<1>(A.c.geo, gi, gj, cls, uu, A.c.fr.s[k], A.c.fr.sinv[k], A.c.md, A.c.qt, e);
#pragma unroll
                    for (int t = 0; t < 9; ++t) E.a[t] += e.a[t];
                }
                if (u == 0 && A.op == OP_HK && gi == gj) {
                    E.a[0].re += 0.5;
                    E.a[4].re += 0.5;
                    E.a[8].re += 0.5;
                }
            }
            sub_residual_share(E, A, fd, d, n, pi, pj, k, u, lpp);
        }
        group_sum(E, lpp);
        if (k < L && u == 0) {
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
        blk Hd = face_block(A.pool, fd[d], n, i, j);
        for (int a = 0; a <= d; ++a) {
            blk F;
#pragma unroll
            for (int q = 0; q < 9; ++q) F.a[q] = Fs[9 * a + q];
            blk HF = blk_mul(Hd, F);
            blk Ha = (a == d) ? Hd : face_block(A.pool, fd[a], n, i, j);
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
    for (int t = 0; t < B.ntile; ++t) {
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
    f.fp32 = B.f32;
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
        atomicAdd((unsigned long long*)&A.st[b].entries, (unsigned long long)max(0, min(TILE, m * n - t * TILE)));
}

// the same pass on one given matrix: out[0] = ACA columns, out[1] = kk
__global__ __launch_bounds__(WG) void k_aca_matrix(char* H, int m, int n, int fp32, double tol, int cap, int kmax,
                                                   double* scratch, int* out)
{
    __shared__ AcaShared S;
    __shared__ RecompShared L;
    AcaWork w = aca_work(scratch, m, n, kmax);
    int kc, kk;
    if (fp32) {
        kc = face_aca_stage((const cx<float>*)H, m, n, w, cap, tol, S);
        kk = face_recompress_stage((cx<float>*)H, m, n, w, kc, tol, L, S);
    } else {
        kc = face_aca_stage((const cx<double>*)H, m, n, w, cap, tol, S);
        kk = face_recompress_stage((cx<double>*)H, m, n, w, kc, tol, L, S);
    }
    if (threadIdx.x == 0) {
        out[0] = kc;
        out[1] = kk;
    }
}

// ---------------------------------------------------------------- compaction

// copy segment q (src offset, dst offset, bytes; offsets 256-aligned, bytes a multiple of 8)
__global__ __launch_bounds__(WG) void k_copy_segments(const char* src, char* dst, const long long* seg, int nseg)
{
    const int q = blockIdx.x;
    if (q >= nseg) return;
    const long long so = seg[3 * q], dof = seg[3 * q + 1], bytes = seg[3 * q + 2];
    const long long n16 = bytes >> 4;
    const uint4* s4 = (const uint4*)(src + so);
    uint4* d4 = (uint4*)(dst + dof);
    for (long long t = threadIdx.x; t < n16; t += WG) d4[t] = s4[t];
    if ((bytes & 8) && threadIdx.x == 0)
        *(unsigned long long*)(dst + dof + 16 * n16) = *(const unsigned long long*)(src + so + 16 * n16);
}

}  // namespace

size_t aca_scratch_doubles(int m, int n, int kmax)
{
    return (size_t)2 * (3 * (size_t)m * kmax + 3 * (size_t)n * kmax + 5 * (size_t)kmax * kmax) + kmax +
           (m + kmax + 4 + 1) / 2 + 8;
}

#define BEM_LAUNCH(kern, grid, block, ...)                                                     \
    do {                                                                                       \
        if ((grid) > 0) hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, st, __VA_ARGS__); \
        BEM_HIP_TRY(hipGetLastError());                                                        \
    } while (0)

void launch_init(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_init, (A.nblocks + 255) / 256, 256, A); }
template <int PATH>
void launch_face_dense_path(const CompressArgs& A, hipStream_t st)
{
    if (A.op == OP_TABLE) BEM_LAUNCH((k_face_dense<2, PATH>), A.nlist, WG, A);
    else if (A.op == OP_V) BEM_LAUNCH((k_face_dense<0, PATH>), A.nlist, WG, A);
    else BEM_LAUNCH((k_face_dense<1, PATH>), A.nlist, WG, A);
}
template <bool F32, bool SELF>
void launch_face_general(const CompressArgs& A, hipStream_t st)
{
    if (A.op == OP_V) BEM_LAUNCH((k_face_general<0, F32, SELF>), A.nlist, WG, A);
    else BEM_LAUNCH((k_face_general<1, F32, SELF>), A.nlist, WG, A);
}
void launch_face_dense(const CompressArgs& A, int path, hipStream_t st)
{
    switch (path) {
        case 0: launch_face_general<false, false>(A, st); break;
        case 1: launch_face_dense_path<1>(A, st); break;
        case 2: launch_face_dense_path<2>(A, st); break;
        case 3: launch_face_general<true, false>(A, st); break;
        case 4: launch_face_general<false, true>(A, st); break;
        default: launch_face_general<true, true>(A, st); break;
    }
}
void launch_face_aca(const CompressArgs& A, hipStream_t st)
{
    BEM_LAUNCH(k_face_aca, A.nlist, WG, A);
    BEM_LAUNCH(k_face_recomp, A.nlist, WG, A);
}
void launch_classify(const DevCtx& c, const BlockIn* blocks, const int* list, const long long* off, int n,
                     unsigned char* cls, hipStream_t st)
{
    BEM_LAUNCH(k_classify, n, WG, c, blocks, list, off, cls);
}
void launch_pivot(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_pivot, (A.nlist + 63) / 64, 64, A); }
void launch_fibre(const CompressArgs& A, hipStream_t st)
{
    BEM_LAUNCH(k_fibre<false>, A.nlist, WG, A);
    BEM_LAUNCH(k_fibre<true>, A.nlist, WG, A);
}
void launch_cross_dense(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_cross_dense, A.nlist, WG, A); }
void launch_final(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_final, (A.nlist + 63) / 64, 64, A); }
void launch_fallback(const CompressArgs& A, int kf, hipStream_t st)
{
    BEM_LAUNCH(k_fallback_alloc, (A.nlist + 63) / 64, 64, A, kf);
}
void launch_fallback_faces(const CompressArgs& A, int kf, hipStream_t st)
{
    BEM_LAUNCH(k_fallback_face, A.nlist, WG, A, kf);
}
void launch_copy_segments(const char* src, char* dst, const long long* seg, int nseg, hipStream_t st)
{
    BEM_LAUNCH(k_copy_segments, nseg, WG, src, dst, seg, nseg);
}
void launch_aca_matrix(char* H, int m, int n, int fp32, double tol, int cap, int kmax, double* scratch, int* out,
                       hipStream_t st)
{
    BEM_LAUNCH(k_aca_matrix, 1, WG, H, m, n, fp32, tol, cap, kmax, scratch, out);
}

}  // namespace bem
