// aca3d.hip -- matrix-valued 3D-ACA (Algorithm 1, Sec. 3) on every block of the
// H-matrix partition, as a pipeline of batched kernels: the host steps the algorithm
// (d = 0, 1, ...) and every phase of a step runs over all blocks still iterating.
//
// Per block, step d:
//   face    H_d[i,j] = ENTRY(i,j,k_d) - sum_{a<d} H_a[i,j] f_a[k_d], every pair generated
//           and stored dense (k_face_dense: regular pairs, one workgroup per 256 pairs;
//           k_face_general: near and self pairs), sigma_3 of each pair reduced per tile;
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
//
// After the last step, the faces of the admissible blocks go through the per-slice ACA as a
// post-pass on the exact stored faces (k_face_aca, one wavefront per face: partial-pivot
// matrix-valued ACA with rank-3 steps and sigma_3 pivots), then the QR + SVD recompression
// of eq. (ACA) (k_face_recomp in recomp.hip).  A face stays dense when its ACA reaches the
// column capacity (unless resumed from a recompression of its columns), when the decay of
// its step norms predicts more columns than 1.5 times the capacity, when it runs out of
// regular pivot rows, or when its factors would not take less memory than the dense face.
// The pivots of the 3D-ACA therefore come from the exact faces: the search of the pivot on
// a reconstruction of the ACA factors, which the paper needs because its faces exist only
// as factors, is not done here.
#include "aca3d.hpp"

namespace bem {

namespace {

constexpr int WG = 256;
constexpr double PIVOT_RTOL = 1e-14;     // matrix-valued ACA of a face: no regular block
// Algorithm 1's "sigma_3 = 0 for all pairs": below this fraction of the block's scale.  A
// residual face formed after d steps carries rounding noise of a few eps times the largest
// face-fibre product subtracted from it, up to about 1e-14 of the scale where the residual's
// 3x3 blocks are all singular; the threshold stays two orders above that noise
constexpr double PIVOT_RTOL_3D = 1e-12;
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

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
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

// Y += H F^H for a 3x3 block H and F = F_{d-1,a} (row-major complex128 in global memory)
__device__ __forceinline__ void acc_hfh(blk& Y, const blk& H, const zd* F)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            zd s = Y.a[3 * i + j];
#pragma unroll
            for (int t = 0; t < 3; ++t) s += mul_conj(H.a[3 * i + t], F[3 * j + t]);
            Y.a[3 * i + j] = s;
        }
}

// Re sum_ij conj(Y_ij) H_ij
__device__ __forceinline__ double re_inner(const blk& Y, const blk& H)
{
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) s += Y.a[q].re * H.a[q].re + Y.a[q].im * H.a[q].im;
    return s;
}

// the share of lane u (of a group of lpp) in the residual of E and in the previous step's
// trace-form terms (sub_residual_cross): faces a = u, u + lpp, ...; every lane adds
// <Y_u, H_{d-1}> for its share Y_u, lane 0 also the t_dd term
__device__ __forceinline__ void sub_residual_share_cross(blk& E, const CompressArgs& A, const FaceDesc* fd,
                                                         const zd* Fb, int d, int n, int i, int j, int k, int u,
                                                         int lpp, double& cross, double& tdd)
{
    blk Y = blk_zero();
    for (int a = u; a < d; a += lpp) {
        const FaceDesc f = fd[a];
        const blk H = face_block(A.pool, f, n, i, j);
        const blk fk = fibre_at(A.pool, f, k);
        blk_mul_sub(E, H, fk);
        if (a < d - 1) acc_hfh(Y, H, Fb + 9 * (size_t)a);
    }
    if (d >= 1) {
        const blk Hp = face_block(A.pool, fd[d - 1], n, i, j);
        cross += re_inner(Y, Hp);
        if (u == 0) {
            blk Z = blk_zero();
            acc_hfh(Z, Hp, Fb + 9 * (size_t)(d - 1));
            tdd += re_inner(Z, Hp);
        }
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
    if (A.sel && !A.sel[b]) return;  // a block of another group of the compression
    BlockState s;
    s.k = 0;
    s.rank = 0;
    s.active = 1;
    s.fallback = 0;
    s.stop = 0;
    s.piv = 0;
    s.nextk = -1;
    s.aca_dense = 0;
    s.term = 0;
    s.aca_cols = 0;
    s.norm2 = 0.0;
    s.hn2 = s.fmax2 = s.s3max = s.fn2 = 0.0;
    s.entries = 0;
    s.recomp_flop = 0.0;
    s.aca_flop = 0.0;
    s.aca_bytes = 0.0;
    s.fref = 0.0;
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

// The trace-form norm terms of the previous step d - 1 at pair (i, j), taken in the
// residual loop of step d while the earlier faces pass through registers (eq. (FrobNorm)):
//   cross += Re sum_{a<d-1} tr(H_a^H H_{d-1} F_{d-1,a}) = Re <sum_a H_a F_{d-1,a}^H, H_{d-1}>
//   tdd   += Re tr(H_{d-1}^H H_{d-1} F_{d-1,d-1})      = Re <H_{d-1} F_{d-1,d-1}^H, H_{d-1}>
// F_{d-1,a} = A.Fda[b][a] as left by the fibre kernel of step d - 1.
template <bool F32>
__device__ __forceinline__ void sub_residual_cross(blk& E, const char* pool, const FaceDesc* fd, const zd* Fb, int d,
                                                   int n, int i, int j, int k, double& cross, double& tdd)
{
    const size_t ld = 3 * (size_t)n;
    blk Y = blk_zero();
#pragma unroll 1
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
        if (a < d - 1) {
            acc_hfh(Y, H, Fb + 9 * (size_t)a);
        } else {
            cross += re_inner(Y, H);
            blk Z = blk_zero();
            acc_hfh(Z, H, Fb + 9 * (size_t)a);
            tdd += re_inner(Z, H);
        }
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
//                [4] cross re, [5] t_dd re, [6] max block |C(k)|^2 of the entries before
//                the residual is taken
// Three waves per SIMD (at most 168 VGPRs, a few spilled): 8 % faster than the two waves
// the compiler's own choice of 176 VGPRs allows
template <int KOP, int PATH>
__global__ __launch_bounds__(WG, 3) void k_face_dense(CompressArgs A)
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
    double s3 = -1.0, e2 = 0.0, cross = 0.0, tdd = 0.0, c2 = 0.0;
    int pi = 0x7fffffff;
    const int i = p / n, j = p - (p / n) * n;
    blk E;
    if (p >= 0) {
        E = pair_entry<KOP, PATH>(A, B.rb + i, B.cb + j, k);
        c2 = blk_fro2(E);
    }
    // the wavefront's largest entry block, reduced before the residual so that the entry
    // block is not kept live through it
    c2 = wave_max(c2);
    if (p >= 0) {
        sub_residual_cross<F32>(E, A.pool, fd, A.Fda + (size_t)b * A.L * 9, d, n, i, j, k, cross, tdd);
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
    double v[3] = {e2, cross, tdd};
    wg_sum<3>(v, S);
    double fm = wg_max(e2, S);
    double cm = wg_max(c2, S);
    wg_argmax(s3, pi, S);
    if (threadIdx.x == 0) {
        double* tp = A.tp + (size_t)(B.tile0 + t) * 8;
        tp[0] = s3;
        tp[1] = (double)pi;
        tp[2] = v[0];
        tp[3] = fm;
        tp[4] = v[1];  // trace-form terms of step d - 1
        tp[5] = v[2];
        tp[6] = cm;
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
    double cross = 0.0, tdd = 0.0, c2 = 0.0;
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
    }
    {
        // the entry before the residual is taken: summed over the lanes of the pair
        blk C = E;
        group_sum(C, lpp);
        if (valid && u == 0) c2 = blk_fro2(C);
        c2 = wave_max(c2);
    }
    if (valid) sub_residual_share_cross(E, A, fd, A.Fda + (size_t)b * A.L * 9, d, n, i, j, k, u, lpp, cross, tdd);
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
    double v[3] = {e2, cross, tdd};
    wg_sum<3>(v, S);
    double fm = wg_max(e2, S);
    double cm = wg_max(c2, S);
    wg_argmax(s3, pi, S);
    if (threadIdx.x == 0) {
        double* tp = A.tp + (size_t)(B.tile0 + t) * 8;
        tp[0] = s3;
        tp[1] = (double)pi;
        tp[2] = v[0];
        tp[3] = fm;
        tp[4] = v[1];  // trace-form terms of step d - 1
        tp[5] = v[2];
        tp[6] = cm;
        atomicAdd((unsigned long long*)&A.st[b].entries, (unsigned long long)max(0, min(ppt, cnt - tl * ppt)));
    }
    (void)m;
}

// Pair order of block list[q]: its pairs p = i cs + j sorted by class (regular, near 1, near
// 2, self), increasing p within a class (a stable partition), written to order[off[q] ..];
// counts[4 q + c] = pairs of class c.  One workgroup per listed block: a counting pass, then
// a scatter pass over chunks of WG pairs with wavefront ballots for the ranks.
__global__ __launch_bounds__(WG) void k_classify(DevCtx c, const BlockIn* blocks, const int* list,
                                                 const long long* off, int* order, int* counts)
{
    __shared__ int cnt[4];
    __shared__ int wcnt[WG / 64][4];
    const BlockIn B = blocks[list[blockIdx.x]];
    const int mn = B.rs * B.cs;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x < 4) cnt[threadIdx.x] = 0;
    __syncthreads();
    int own[4] = {0, 0, 0, 0};
    for (int p = threadIdx.x; p < mn; p += WG) {
        const int i = p / B.cs, j = p - i * B.cs;
        ++own[pair_class(c.geo, B.rb + i, B.cb + j, c.qt)];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) atomicAdd(&cnt[k], own[k]);
    __syncthreads();
    int base[4];
    base[0] = 0;
    base[1] = cnt[0];
    base[2] = cnt[0] + cnt[1];
    base[3] = cnt[0] + cnt[1] + cnt[2];
    if (threadIdx.x < 4) counts[4 * (size_t)blockIdx.x + threadIdx.x] = cnt[threadIdx.x];
    int* o = order + off[blockIdx.x];
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int p0 = 0; p0 < mn; p0 += WG) {
        const int p = p0 + threadIdx.x;
        int k = -1;
        if (p < mn) {
            const int i = p / B.cs, j = p - i * B.cs;
            k = pair_class(c.geo, B.rb + i, B.cb + j, c.qt);
        }
        int rank = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const unsigned long long m = __ballot(k == q);
            if (k == q) rank = __popcll(m & below);
            if (lane == 0) wcnt[wv][q] = __popcll(m);
        }
        __syncthreads();
        if (k >= 0) {
            int pos = base[k] + rank;
            for (int w = 0; w < wv; ++w) pos += wcnt[w][k];
            o[pos] = p;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            for (int w = 0; w < WG / 64; ++w) base[q] += wcnt[w][q];
        __syncthreads();
    }
}

// ---------------------------------------------------------------- per-slice ACA of far faces

struct AcaShared {
    Red r;
    zd pinv[9];
    double s;
    int piv, flag;
};

// ---------------------------------------------------------------- per-slice ACA
//
// One wavefront per face: a lane per block column (row pass) or block row (column pass),
// wavefront reductions, no LDS.  The ACA is bound by the latency of reading the stored face
// and the earlier columns, so many faces per CU (small register footprint) beat many lanes
// per face: k_face_aca asks for four waves per SIMD (128 VGPRs; left to itself the compiler
// takes 255 and runs one), 15 % faster on the metric's workload.
constexpr int WA = 64;
constexpr int KMAX_SLICE = 96;  // largest ACA column count (the scratch and LDS capacity)
constexpr int CB = 8;           // earlier ACA columns read per batch in the residual passes

__device__ __forceinline__ double wmax(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// a wavefront-uniform double moved to scalar registers
__device__ __forceinline__ double uniform_d(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b), hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// sigma_3 of a block as a call: its eigenvalue solve (acos, cos) is the register peak of the
// ACA loop, and a call keeps it out of the loop's allocation
__device__ __noinline__ double sigma3_call(const blk E) { return blk_sigma3_scaled(E); }

// argmax over the wavefront with ties to the smallest index; NaN counts as -inf
__device__ __forceinline__ void wargmax(double& v, int& idx)
{
    if (!(v == v)) v = -1.0;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double ov = __shfl_xor(v, o, 64);
        const int oi = __shfl_xor(idx, o, 64);
        if (ov > v || (ov == v && oi < idx)) {
            v = ov;
            idx = oi;
        }
    }
}

// Matrix-valued partial-pivot ACA of the stored face with rank-3 steps and sigma_3 pivots
// (the matrix form of the pivoting of Algorithm 1).  Stops once the newest 3 columns satisfy
// ||U_k||_F ||V_k||_F <= tol, or when a residual row without a regular block is itself
// below tol.  Returns the number of columns, or -1 when the face is not resolved within cap
// columns short of 3 min(m, n) (or MAX_FAIL rows in a row have no regular pivot, or a row
// skipped that way is left at the end): the caller keeps the face dense.
//
// One wavefront.  The residual passes give a lane one scalar column (row pass) or one scalar
// row (column pass) of the pivot block row / column, so that the reads of the earlier ACA
// columns are contiguous across lanes; the pivot's own 3 x kc slice is staged in LDS (sk).
// The sigma_3 pivot search then reads the stored 3 x 3 blocks back.
//
// kc0 > 0 resumes a run with kc0 columns already in U, V (recompressed from an earlier run that
// reached the column capacity) at row irow0, with the used rows of that run.  resumable: on
// reaching cap short of 3 min(m, n) columns the run returns -2 (and the next row in
// info[2]) instead of -1, for the caller to recompress and resume.
//
// abort > 0 (the compression pass without resume): once ABORT_STEPS rank-3 steps are done, the
// decay of the step norms ||U_k|| ||V_k|| so far is extrapolated geometrically; a face whose
// predicted column count to reach tol exceeds abort * cap is given up (-1, kept dense) without
// running to the cap.  Such faces would mostly end dense anyway, and every further step re-reads
// all earlier columns.  abort = 0 keeps the plain stopping rules.
constexpr int ABORT_STEPS = 8;
constexpr double ACA_ABORT = 1.5;

// Growth of ||S||_F^2, S = U V^H, when the columns kc .. kc + 2 join the kc earlier ones:
// 2 Re sum_{c < kc} sum_x (u_c^H u_x)(v_x^H v_c) + sum_{y, x} (u_y^H u_x)(v_x^H v_y) over the
// new columns x, y (one wavefront).
__device__ double aca_norm_growth(const AcaWork& w, int M3, int N3, int kc)
{
    double g = 0.0;
    for (int c = 0; c < kc + 3; ++c) {
        double a[12];
#pragma unroll
        for (int t = 0; t < 12; ++t) a[t] = 0.0;
        const zd* uc = w.U + (size_t)c * M3;
        for (int q = threadIdx.x; q < M3; q += WA) {
            const zd u = uc[q];
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                const zd t = conj_mul(u, w.U[(size_t)(kc + x) * M3 + q]);
                a[2 * x] += t.re;
                a[2 * x + 1] += t.im;
            }
        }
        const zd* vc = w.V + (size_t)c * N3;
        for (int q = threadIdx.x; q < N3; q += WA) {
            const zd v = vc[q];
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                const zd t = conj_mul(w.V[(size_t)(kc + x) * N3 + q], v);
                a[6 + 2 * x] += t.re;
                a[7 + 2 * x] += t.im;
            }
        }
#pragma unroll
        for (int t = 0; t < 12; ++t) a[t] = wsum(a[t]);
        double r = 0.0;
#pragma unroll
        for (int x = 0; x < 3; ++x) r += a[2 * x] * a[6 + 2 * x] - a[2 * x + 1] * a[7 + 2 * x];
        g += (c < kc ? 2.0 : 1.0) * r;
    }
    return g;
}

template <typename T>
__device__ int face_aca(const cx<T>* H, int m, int n, const AcaWork& w, int cap, double tol, double amax, zd* pinv,
                        zd* sk, int kc0, int irow0, bool resumable, double abort, int& built,
                        double rel = 0.0)
{
    double s2n = 0.0;  // ||U V^H||_F^2 of the columns so far (rel > 0)
    double est0 = 0.0;
    const int lane = threadIdx.x;
    const int M3 = 3 * m, N3 = 3 * n;
    if (kc0 == 0)
        for (int i = lane; i < m; i += WA) w.usedrow[i] = 0;
    __syncthreads();
    int kc = kc0, fails = 0, skipped = 0, irow = irow0;
    built = kc0;
    for (;;) {
        if (kc + 3 > cap) {
            if (kc >= 3 * min(m, n)) return kc;  // all of min(m, n) interpolated: exact
            if (!resumable) return -1;
            if (lane == 0) w.info[2] = irow;
            return -2;
        }
        // residual row block irow -> V columns kc..kc+2 (row^H); sk = U rows 3 irow .. + 2
        for (int q = lane; q < 3 * kc; q += WA) {
            const int c = q / 3, y = q - 3 * c;
            sk[q] = w.U[(size_t)c * M3 + 3 * irow + y];
        }
        __syncthreads();
        double rn2 = 0.0;
        for (int q = lane; q < N3; q += WA) {
            zd e[3];
#pragma unroll
            for (int y = 0; y < 3; ++y) e[y] = ldz(H + (size_t)(3 * irow + y) * N3 + q);
            const zd* vq = w.V + q;
            int c = 0;
            for (; c + CB <= kc; c += CB) {  // CB loads in flight per lane
                zd v[CB];
#pragma unroll
                for (int t = 0; t < CB; ++t) v[t] = vq[(size_t)(c + t) * N3];
#pragma unroll
                for (int t = 0; t < CB; ++t)
#pragma unroll
                    for (int y = 0; y < 3; ++y) e[y] -= mul_conj(sk[3 * (c + t) + y], v[t]);
            }
            for (; c < kc; ++c) {
                const zd v = vq[(size_t)c * N3];
#pragma unroll
                for (int y = 0; y < 3; ++y) e[y] -= mul_conj(sk[3 * c + y], v);
            }
#pragma unroll
            for (int y = 0; y < 3; ++y) {
                w.V[(size_t)(kc + y) * N3 + q] = conj(e[y]);
                rn2 += abs2(e[y]);
            }
        }
        if (lane == 0) w.usedrow[irow] = 1;
        rn2 = wsum(rn2);
        __syncthreads();
        double best = -1.0;
        int bj = 0x7fffffff;
        for (int j = lane; j < n; j += WA) {
            blk E;
#pragma unroll
            for (int y = 0; y < 3; ++y)
#pragma unroll
                for (int x = 0; x < 3; ++x) E.a[3 * y + x] = conj(w.V[(size_t)(kc + y) * N3 + 3 * j + x]);
            const double s3 = sigma3_call(E);
            if (s3 > best || (s3 == best && j < bj)) {
                best = s3;
                bj = j;
            }
        }
        wargmax(best, bj);
        if (!(best > PIVOT_RTOL * amax)) {
            if (sqrt(rn2) <= fmax(tol, rel * sqrt(fmax(s2n, 0.0)))) return kc;  // negligible residual row
            ++skipped;
            if (++fails >= MAX_FAIL) return -1;
            int cand = 0x7fffffff;
            for (int i = lane; i < m; i += WA)
                if (!w.usedrow[i] && i < cand) cand = i;
            double cv = cand == 0x7fffffff ? -1.0 : 1.0;
            wargmax(cv, cand);
            if (cv < 0.0) return -1;  // every row visited, a skipped row remains
            irow = cand;
            __syncthreads();
            continue;
        }
        fails = 0;
        // pivot block P = residual block (irow, bj), its inverse shared through LDS; sk = V
        // rows 3 bj .. + 2
        if (lane == 0) {
            blk P;
#pragma unroll
            for (int y = 0; y < 3; ++y)
#pragma unroll
                for (int x = 0; x < 3; ++x) P.a[3 * y + x] = conj(w.V[(size_t)(kc + y) * N3 + 3 * bj + x]);
            const blk Pi = blk_inv(P);
#pragma unroll
            for (int t = 0; t < 9; ++t) pinv[t] = Pi.a[t];
        }
        for (int q = lane; q < 3 * kc; q += WA) {
            const int c = q / 3, x = q - 3 * c;
            sk[q] = w.V[(size_t)c * N3 + 3 * bj + x];
        }
        __syncthreads();
        zd pv[9];  // P^{-1}, uniform: kept in scalar registers
#pragma unroll
        for (int t = 0; t < 9; ++t) pv[t] = {uniform_d(pinv[t].re), uniform_d(pinv[t].im)};
        // residual column block bj -> U columns kc..kc+2 = column * P^{-1}
        double un2 = 0.0;
        for (int q = lane; q < M3; q += WA) {
            zd e[3];
#pragma unroll
            for (int x = 0; x < 3; ++x) e[x] = ldz(H + (size_t)q * N3 + 3 * bj + x);
            const zd* uq = w.U + q;
            int c = 0;
            for (; c + CB <= kc; c += CB) {
                zd u[CB];
#pragma unroll
                for (int t = 0; t < CB; ++t) u[t] = uq[(size_t)(c + t) * M3];
#pragma unroll
                for (int t = 0; t < CB; ++t)
#pragma unroll
                    for (int x = 0; x < 3; ++x) e[x] -= mul_conj(u[t], sk[3 * (c + t) + x]);
            }
            for (; c < kc; ++c) {
                const zd u = uq[(size_t)c * M3];
#pragma unroll
                for (int x = 0; x < 3; ++x) e[x] -= mul_conj(u, sk[3 * c + x]);
            }
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                zd t = e[0] * pv[x];
                t = fma_c(e[1], pv[3 + x], t);
                t = fma_c(e[2], pv[6 + x], t);
                w.U[(size_t)(kc + x) * M3 + q] = t;
                un2 += abs2(t);
            }
        }
        un2 = wsum(un2);
        double thr = tol;
        if (rel > 0.0) {
            // the stop of the ACA relative to the approximation so far (rel ||U V^H||_F)
            __syncthreads();
            s2n += aca_norm_growth(w, M3, N3, kc);
            thr = fmax(tol, rel * sqrt(fmax(s2n, 0.0)));
        }
        kc += 3;
        built = kc;
        const double est = sqrt(un2 * rn2);
        if (est <= thr) return kc;
        if (kc == 3) est0 = est;
        if (abort > 0.0 && kc >= 3 * ABORT_STEPS && est0 > 0.0) {
            const double rate = pow(est / est0, 3.0 / (kc - 3));  // per step
            const double steps = rate < 1.0 ? log(tol / est) / log(rate) : 1e30;
            if (kc + 3.0 * steps > abort * cap) return -1;
        }
        __syncthreads();
        double best2 = -1.0;
        int bi2 = 0x7fffffff;
        for (int i = lane; i < m; i += WA) {
            if (w.usedrow[i]) continue;
            blk Un;
#pragma unroll
            for (int y = 0; y < 3; ++y)
#pragma unroll
                for (int x = 0; x < 3; ++x) Un.a[3 * y + x] = w.U[(size_t)(kc - 3 + x) * M3 + 3 * i + y];
            const double s3 = sigma3_call(Un);
            if (s3 > best2 || (s3 == best2 && i < bi2)) {
                best2 = s3;
                bi2 = i;
            }
        }
        wargmax(best2, bi2);
        if (best2 < 0.0) return skipped ? -1 : kc;  // every row is a pivot row: exact
        irow = bi2;
        __syncthreads();
    }
}

// ACA stage of one stored dense face: ||H||_F, the pivot scale max |H|, then face_aca;
// returns the column count (-1: not resolved, or a zero face).  One wavefront.
template <typename T>
__device__ int face_aca_stage(const cx<T>* H, int m, int n, const AcaWork& w, int cap, double tol, int kc0, int irow0,
                              bool resumable, double abort, int& built, double rel = 0.0)
{
    double s2 = 0.0, amax = 0.0;
    const int cnt = 9 * m * n;
    for (int q = threadIdx.x; q < cnt; q += WA) {
        const double a2 = abs2(ldz(H + q));
        s2 += a2;
        amax = fmax(amax, a2);
    }
    s2 = wsum(s2);
    amax = sqrt(wmax(amax));
    __shared__ zd pinv[9];
    __shared__ zd sk[3 * KMAX_SLICE];
    if (cap > KMAX_SLICE) return -1;
    return s2 > 0.0 ? face_aca(H, m, n, w, cap, tol, amax, pinv, sk, kc0, irow0, resumable, abort, built, rel) : -1;
}

// Absolute tolerance of face d of block b: eps_aca ||C^(r)||_F / ||f_d||_F, so that each
// face-fibre term errs by at most about eps_aca ||C^(r)||_F.  One wavefront.
__device__ double face_tol(const CompressArgs& A, int b, const FaceDesc& f)
{
    double fn2 = 0.0;
    const zd* fib = (const zd*)(A.pool + f.fib_off);
    for (int q = threadIdx.x; q < 9 * A.L; q += WA) fn2 += abs2(fib[q]);
    fn2 = wsum(fn2);
    return fn2 > 0.0 ? A.eps_aca_far * sqrt(fmax(A.st[b].norm2, 0.0) / fn2) : 0.0;
}

// Per-slice ACA pass, one wavefront per listed face (items (block << 8) | d, scratch slot =
// position in the list): k_face_aca leaves the ACA columns, their count and the face's
// tolerance in the slot; k_face_recomp (recomp.hip) recompresses them and rewrites the face
// descriptor.  A run that reaches the column capacity of the slot (KMAX_SLICE) on a face whose
// factors could still save memory returns -2: k_face_recomp recompresses its columns into the
// slot's other half at a tighter tolerance and leaves state -3, and a resume launch
// (resume = 1) continues the run from those columns.
__global__ __launch_bounds__(WA, 4) void k_face_aca(CompressArgs A, int resume)
{
    const int item = A.list[blockIdx.x];
    const int b = item >> 8, d = item & 255;
    const BlockIn B = A.blocks[b];
    const FaceDesc f = A.faces[(size_t)b * A.L + d];
    const int m = B.rs, n = B.cs;
    AcaWork w = aca_work(A.scratch + A.slot_off[blockIdx.x], m, n, A.kmax, ACA_HALVES);
    if (resume && w.info[0] != -3) return;
    if (A.iloop) {
        // a face of the current 3D-ACA step (Sec. 3.1 order): relative tolerance, no resume,
        // no early end; blocks that ended at this step are left alone (state 0)
        int kc = 0, built = 0;
        if (A.st[b].active && f.kk == 0 && !f.sel) {
            const int cap = min(A.kmax, face_aca_cap(m, n));
            kc = f.fp32 ? face_aca_stage((const cx<float>*)(A.pool + f.face_off), m, n, w, cap, 0.0, 0, 0, false, 0.0,
                                         built, A.eps_aca_far)
                        : face_aca_stage((const cx<double>*)(A.pool + f.face_off), m, n, w, cap, 0.0, 0, 0, false, 0.0,
                                         built, A.eps_aca_far);
        }
        if (threadIdx.x == 0) {
            w.info[0] = kc;
            w.info[3] = 0;
            w.tol[0] = 0.0;
            const double t1 = built / 3, mn = (double)(m + n);
            if (t1 > 0) {
                // as below, plus the norm growth: 3 (m + n) (3t + 3) complex multiply-adds per step
                atomicAdd(&A.st[b].aca_flop, 8.0 * (13.5 * mn * t1 * (t1 - 1.0) + 27.0 * m * t1 +
                                                    4.5 * mn * t1 * (t1 + 1.0) + 9.0 * mn * t1));
                atomicAdd(&A.st[b].aca_bytes, 72.0 * mn * t1 * (t1 - 1.0) * 2.0 +
                                                  t1 * (9.0 * mn * (f.fp32 ? 8.0 : 16.0) + 144.0 * mn));
            }
        }
        return;
    }
    int kc = -1, built = 0, kc0 = 0, irow0 = 0;
    double tol = 0.0;
    if (resume) {
        kc0 = w.info[1];
        irow0 = w.info[2];
        tol = w.tol[0];
        aca_select_half(w);
    } else if (threadIdx.x == 0) {
        w.info[3] = 0;
    }
    if (f.kk == 0 && !f.sel) {
        const int cap = min(A.kmax, face_aca_cap(m, n));
        const bool resumable = A.aca_rounds > 0 && cap == KMAX_SLICE && face_aca_cap(m, n) > KMAX_SLICE;
        const double abort = A.aca_rounds > 0 ? 0.0 : ACA_ABORT;
        if (!resume) tol = face_tol(A, b, f);
        kc = f.fp32 ? face_aca_stage((const cx<float>*)(A.pool + f.face_off), m, n, w, cap, tol, kc0, irow0, resumable,
                                     abort, built)
                    : face_aca_stage((const cx<double>*)(A.pool + f.face_off), m, n, w, cap, tol, kc0, irow0, resumable,
                                     abort, built);
    }
    if (threadIdx.x == 0) {
        w.info[0] = kc;
        w.tol[0] = tol;
        if (kc == -2) w.info[1] = built;  // the columns to recompress
        // algorithmic work of the rank-3 steps t = t0 .. t1 - 1 of this run (t0 = kc0 / 3,
        // t1 = built / 3): step t updates a 3-row and a 3-column block by the 3t earlier columns
        // (9 (m + n) 3t complex multiply-adds, reading 3 (m + n) 3t earlier column entries in
        // FP64) and scales the new columns by the pivot inverse (27 m); it reads 9 (m + n) face
        // entries and writes 9 (m + n) column entries
        const double t0 = kc0 / 3, t1 = built / 3, mn = (double)(m + n);
        const double tri = t1 * (t1 - 1.0) - t0 * (t0 - 1.0);
        const double macs = 13.5 * mn * tri + 27.0 * m * (t1 - t0);
        const double bytes = 72.0 * mn * tri + (t1 - t0) * (9.0 * mn * (f.fp32 ? 8.0 : 16.0) + 144.0 * mn);
        if (t1 > t0) {
            atomicAdd(&A.st[b].aca_flop, 8.0 * macs);
            atomicAdd(&A.st[b].aca_bytes, bytes);
        }
    }
}

// ---------------------------------------------------------------- faces inside the loop

// After k_face_recomp in the in-loop order: the factors of each listed face (slot state -5,
// complex128 column-major in the slot's second half) move to the pool in the face's
// precision, Ubar (3m x kk) then Vbar (3n x kk), row-major; fac_kk = 0 for a face that stays
// exact.  One workgroup per listed face.
__global__ __launch_bounds__(WG) void k_iloop_store(CompressArgs A)
{
    __shared__ long long off_s;
    const int item = A.list[blockIdx.x];
    const int b = item >> 8, d = item & 255;
    const BlockIn B = A.blocks[b];
    const int m = B.rs, n = B.cs;
    const size_t fi = (size_t)b * A.L + d;
    AcaWork w = aca_work(A.scratch + A.slot_off[blockIdx.x], m, n, A.kmax, ACA_HALVES);
    const int state = w.info[0];
    const int kk = w.info[1];
    if (state != -5 || kk <= 0) {
        if (threadIdx.x == 0) A.fac_kk[fi] = 0;
        return;
    }
    const FaceDesc f = A.faces[fi];
    if (threadIdx.x == 0) off_s = pool_alloc(A, (long long)(f.fp32 ? sizeof(zf) : sizeof(zd)) * 3 * (m + n) * kk);
    __syncthreads();
    const long long off = off_s;
    if (off < 0) {  // pool exhausted (the error flag is set): the face stays exact
        if (threadIdx.x == 0) A.fac_kk[fi] = 0;
        return;
    }
    const zd* U2 = w.U2;
    const zd* V2 = w.V2;
    const int M3 = 3 * m, N3 = 3 * n;
    for (int q = threadIdx.x; q < (M3 + N3) * kk; q += WG) {
        const int r = q / kk, c = q - r * kk;
        const zd v = r < M3 ? U2[(size_t)c * M3 + r] : V2[(size_t)c * N3 + (r - M3)];
        if (f.fp32) stz((zf*)(A.pool + off) + q, v);
        else ((zd*)(A.pool + off))[q] = v;
    }
    if (threadIdx.x == 0) {
        A.fac_off[fi] = off;
        A.fac_kk[fi] = kk;
        atomicAdd((unsigned long long*)&A.st[b].aca_cols, (unsigned long long)w.info[2]);
    }
}

// The pivot search of Sec. 3.1 on the reconstruction: for every pair (i, j) of an in-loop
// face with factors, H[i,j] = Ubar[3i..3i+2] Vbar[3j..3j+2]^H from the stored factors is
// written over the exact face (the later residuals, the fibre and the norm use it), and the
// tile partials of k_pivot (sigma_3 argmax, ||H||_F^2, max block norm) are those of the
// reconstruction.  Items (block << 12) | t for every face tile t of the block: tiles of
// TILE consecutive pairs p = i n + j up to m n, the others neutral.
__global__ __launch_bounds__(WG) void k_iloop_recon(CompressArgs A)
{
    __shared__ Red S;
    const int item = A.list[blockIdx.x];
    const int b = item >> 12, t = item & 4095;
    if (!A.st[b].active) return;
    const BlockIn B = A.blocks[b];
    const int m = B.rs, n = B.cs, d = A.d;
    const size_t fi = (size_t)b * A.L + d;
    const int kk = A.fac_kk[fi];
    if (kk <= 0) return;  // the exact face and its partials stand
    const FaceDesc F = A.faces[fi];
    const int p = t * TILE + threadIdx.x;
    double s3 = -1.0, e2 = 0.0;
    int pi = 0x7fffffff;
    if (p < m * n) {
        const int i = p / n, j = p - (p / n) * n;
        blk H;
#pragma unroll
        for (int q = 0; q < 9; ++q) H.a[q] = {0.0, 0.0};
        const size_t ld = 3 * (size_t)n;
        if (F.fp32) {
            const zf* Ub = (const zf*)(A.pool + A.fac_off[fi]);
            const zf* Vb = Ub + (size_t)3 * m * kk;
            for (int r = 0; r < kk; ++r) {
                zd u[3], v[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    u[a] = ldz(Ub + (size_t)(3 * i + a) * kk + r);
                    v[a] = ldz(Vb + (size_t)(3 * j + a) * kk + r);
                }
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int c = 0; c < 3; ++c) H.a[3 * a + c] += mul_conj(u[a], v[c]);
            }
            zf* Hd = (zf*)(A.pool + F.face_off);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const zf wv = {(float)H.a[3 * a + c].re, (float)H.a[3 * a + c].im};
                    Hd[(size_t)(3 * i + a) * ld + 3 * j + c] = wv;
                    H.a[3 * a + c] = {(double)wv.re, (double)wv.im};  // search on the stored face
                }
        } else {
            const zd* Ub = (const zd*)(A.pool + A.fac_off[fi]);
            const zd* Vb = Ub + (size_t)3 * m * kk;
            for (int r = 0; r < kk; ++r) {
                zd u[3], v[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    u[a] = Ub[(size_t)(3 * i + a) * kk + r];
                    v[a] = Vb[(size_t)(3 * j + a) * kk + r];
                }
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int c = 0; c < 3; ++c) H.a[3 * a + c] += mul_conj(u[a], v[c]);
            }
            zd* Hd = (zd*)(A.pool + F.face_off);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) Hd[(size_t)(3 * i + a) * ld + 3 * j + c] = H.a[3 * a + c];
        }
        e2 = blk_fro2(H);
        s3 = blk_sigma3_scaled(H);
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
        tp[6] = fm;  // the slice itself is never formed: its reconstructed residual stands in
    }
}

// After the last step: the in-loop faces of a block (not a dense fallback) that kept factors
// are stored as factors; their reconstructions are dropped by the compaction.
__global__ __launch_bounds__(64) void k_iloop_finish(CompressArgs A)
{
    const int q = blockIdx.x * 64 + threadIdx.x;
    if (q >= A.nlist) return;
    const int b = A.list[q];
    const BlockState s = A.st[b];
    if (s.fallback) return;
    int dense = 0;
    for (int d = 0; d < s.rank; ++d) {
        const size_t fi = (size_t)b * A.L + d;
        FaceDesc f = A.faces[fi];
        if (f.kk != 0 || f.sel) continue;
        if (A.fac_kk[fi] > 0) {
            f.face_off = A.fac_off[fi];
            f.kk = A.fac_kk[fi];
            A.faces[fi] = f;
        } else {
            ++dense;
        }
    }
    A.st[b].aca_dense += dense;
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
    double best = -1.0, h2 = 0.0, fm = 0.0, cm = 0.0;
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
        cm = fmax(cm, tp[6]);
    }
    s.hn2 = h2;
    s.fmax2 = fm;
    s.s3max = best;
    s.stop = 0;
    // the scale of the pivot test: the block's magnitude, the largest 3x3 block of the
    // slices C(k_1..k_d) formed so far.  A pivot judged against the shrinking residual face,
    // or against a slice smaller than a later one, lets rounding noise of a residual of
    // rank-deficient 3 x 3 blocks through as a pivot
    s.fref = fmax(s.fref, sqrt(cm));
    const double eps = block_eps(A, B);
    if (d > 0 && sqrt(h2) <= eps * sqrt(fmax(s.norm2, 0.0))) {
        // the residual face vanishes: C^(d-1) reproduces the array; rank d
        s.stop = 1;
        s.active = 0;
        s.rank = d;
    } else if (!(best > PIVOT_RTOL_3D * s.fref)) {
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
template <int KOP, bool GEN>
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
        const bool gen = KOP != 2 && pair_class(A.c.geo, B.rb + pi, B.cb + pj, A.c.qt) != CLS_REGULAR;
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
    // regular rule: the entry on the first lane of a group, the residual over the earlier
    // faces shared by the group's lanes (as many as the L frequencies leave in the workgroup)
    int lpp = pair_lanes(cls);
    if (!GEN)
        while (lpp < 64 && 2 * lpp * L <= WG) lpp *= 2;
    const int nu = GEN ? rule_units(cls, A.c.qt) : 1;
    const int u = threadIdx.x % lpp;
    for (int k0 = 0; k0 < L; k0 += WG / lpp) {
        const int k = k0 + threadIdx.x / lpp;
        blk E = blk_zero();
        if (k < L) {
            if constexpr (KOP == 2) {
                if (u == 0) E = entry_dispatch<false>(A.c, OP_TABLE, gi, gj, k);
            } else if constexpr (!GEN) {
                if (u == 0) {
                    if (B.f32) entry_regular<float>(A.c.geo, KOP, gi, gj, A.c.fr.sf[k], A.c.fr.sinvf[k], A.c.mf, E);
                    else entry_regular<double>(A.c.geo, KOP, gi, gj, A.c.fr.s[k], A.c.fr.sinv[k], A.c.md, E);
                }
            } else {
                for (int uu = u; uu < nu; uu += lpp) {
                    blk e;
                    entry_unit<KOP>(A.c.geo, gi, gj, cls, uu, A.c.fr.s[k], A.c.fr.sinv[k], A.c.md, A.c.qt, e);
#pragma unroll
                    for (int t = 0; t < 9; ++t) E.a[t] += e.a[t];
                }
                if (u == 0 && KOP == 1 && gi == gj) {
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
    // F_da = sum_k f_d[k] f_a[k]^H for a <= d: one wavefront per face a, its lanes over k,
    // a wavefront reduction each (no workgroup barrier per face)
    {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        for (int a = w; a <= d; a += WG / 64) {
            double Fv[18];
#pragma unroll
            for (int t = 0; t < 18; ++t) Fv[t] = 0.0;
            const zd* fa = (const zd*)(A.pool + fd[a].fib_off);
            for (int k = lane; k < L; k += 64) {
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
#pragma unroll
            for (int t = 0; t < 18; ++t) Fv[t] = wsum(Fv[t]);
            if (lane == 0)
                for (int t = 0; t < 9; ++t) A.Fda[((size_t)b * L + a) * 9 + t] = {Fv[2 * t], Fv[2 * t + 1]};
        }
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
    if (!A.st[b].active || A.st[b].stop || !A.st[b].term) return;
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

// Step d of a block that has no next frequency (d + 1 == L or every k used): its trace-form
// terms come from k_cross_dense; norm update and the test of eq. (precision).
__global__ __launch_bounds__(64) void k_final(CompressArgs A)
{
    int q = blockIdx.x * 64 + threadIdx.x;
    if (q >= A.nlist) return;
    const int b = A.list[q];
    BlockState s = A.st[b];
    if (!s.active || s.stop || !s.term) return;
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
    s.rank = !(sqrt(s.hn2 * s.fn2) > eps * sqrt(fmax(s.norm2, 0.0))) ? d : d + 1;  // sub-tolerance pair dropped
    s.active = 0;
    A.st[b] = s;
}

// After the fibre of step d: a block with a next frequency starts step d + 1 before the test
// of step d is known (its trace-form terms come with the face kernels of step d + 1);
// without one it is terminal (k_cross_dense, k_final).
__global__ __launch_bounds__(64) void k_advance(CompressArgs A)
{
    int q = blockIdx.x * 64 + threadIdx.x;
    if (q >= A.nlist) return;
    const int b = A.list[q];
    BlockState s = A.st[b];
    if (!s.active || s.stop) return;
    const int d = A.d;
    if (s.nextk < 0 || d + 1 == A.L) {
        s.term = 1;
    } else {
        s.k = s.nextk;
        if (!alloc_step(A, b, d + 1, s.k)) {
            s.term = 1;  // pool exhausted: the error flag is set, the block ends here
        }
    }
    A.st[b] = s;
}

// After the face kernels of step d (d >= 1): trace-form terms of step d - 1 (tile partials
// 4, 5), norm update and the test of eq. (precision) for step d - 1.  On failure the pair
// d - 1 is dropped (rank d - 1) and the face of step d is discarded.
__global__ __launch_bounds__(64) void k_final_prev(CompressArgs A)
{
    int q = blockIdx.x * 64 + threadIdx.x;
    if (q >= A.nlist) return;
    const int b = A.list[q];
    BlockState s = A.st[b];
    if (!s.active) return;
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
        s.rank = d - 1;
        s.active = 0;
        s.entries -= (long long)B.rs * B.cs;  // the face of step d is not kept
    } else {
        s.rank = d;
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

// the ACA stage on one given matrix: out[0] = ACA columns (the recompression follows in
// k_aca_matrix_recomp, which sets out[1])
__global__ __launch_bounds__(WA) void k_aca_matrix(char* H, int m, int n, int fp32, double tol, int cap, int kmax,
                                                   double* scratch, int* out)
{
    AcaWork w = aca_work(scratch, m, n, kmax);
    int built = 0;
    const int kc = fp32 ? face_aca_stage((const cx<float>*)H, m, n, w, cap, tol, 0, 0, false, 0.0, built)
                        : face_aca_stage((const cx<double>*)H, m, n, w, cap, tol, 0, 0, false, 0.0, built);
    if (threadIdx.x == 0) {
        out[0] = kc;
        out[1] = 0;
        w.info[0] = kc;
        w.tol[0] = tol;
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

size_t aca_scratch_doubles(int m, int n, int kmax, int halves)
{
    return (size_t)2 * (3 * (size_t)halves * m * kmax + 3 * (size_t)halves * n * kmax + 5 * (size_t)kmax * kmax) +
           kmax + (m + kmax + 4 + 1) / 2 + 8;
}

#define BEM_LAUNCH(kern, grid, block, ...)                                                     \
    do {                                                                                       \
        if ((grid) > 0) hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, st, __VA_ARGS__); \
        BEM_HIP_TRY(hipGetLastError());                                                        \
    } while (0)

void launch_init(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_init, (A.nblocks + 255) / 256, 256, A); }
void launch_iloop_store(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_iloop_store, A.nlist, WG, A); }
void launch_iloop_recon(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_iloop_recon, A.nlist, WG, A); }
void launch_iloop_finish(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_iloop_finish, (A.nlist + 63) / 64, 64, A); }
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
void launch_face_aca(const CompressArgs& A, hipStream_t st, int resume)
{
    BEM_LAUNCH(k_face_aca, A.nlist, WA, A, resume);
}
void launch_classify(const DevCtx& c, const BlockIn* blocks, const int* list, const long long* off, int n,
                     int* order, int* counts, hipStream_t st)
{
    BEM_LAUNCH(k_classify, n, WG, c, blocks, list, off, order, counts);
}
void launch_pivot(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_pivot, (A.nlist + 63) / 64, 64, A); }
void launch_fibre(const CompressArgs& A, hipStream_t st)
{
    if (A.op == OP_TABLE) {
        BEM_LAUNCH((k_fibre<2, false>), A.nlist, WG, A);
    } else if (A.op == OP_V) {
        BEM_LAUNCH((k_fibre<0, false>), A.nlist, WG, A);
        BEM_LAUNCH((k_fibre<0, true>), A.nlist, WG, A);
    } else {
        BEM_LAUNCH((k_fibre<1, false>), A.nlist, WG, A);
        BEM_LAUNCH((k_fibre<1, true>), A.nlist, WG, A);
    }
}
void launch_cross_dense(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_cross_dense, A.nlist, WG, A); }
void launch_final(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_final, (A.nlist + 63) / 64, 64, A); }

namespace {
// flags[b] = block b still iterating (the host's view of the next step)
__global__ __launch_bounds__(256) void k_active_flags(const BlockState* st, int nb, unsigned char* flags)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b < nb) flags[b] = (unsigned char)(st[b].active != 0);
}
}  // namespace

void launch_active_flags(const CompressArgs& A, unsigned char* flags, hipStream_t st)
{
    hipLaunchKernelGGL(k_active_flags, dim3((A.nblocks + 255) / 256), dim3(256), 0, st, A.st, A.nblocks, flags);
    BEM_HIP_TRY(hipGetLastError());
}
void launch_advance(const CompressArgs& A, hipStream_t st) { BEM_LAUNCH(k_advance, (A.nlist + 63) / 64, 64, A); }
void launch_final_prev(const CompressArgs& A, hipStream_t st)
{
    BEM_LAUNCH(k_final_prev, (A.nlist + 63) / 64, 64, A);
}
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
    BEM_LAUNCH(k_aca_matrix, 1, WA, H, m, n, fp32, tol, cap, kmax, scratch, out);
    launch_aca_matrix_recomp(H, m, n, fp32, kmax, scratch, out, st);
}

}  // namespace bem
