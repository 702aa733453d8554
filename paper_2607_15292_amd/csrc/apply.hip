// apply.hip -- transposed products and the gCQ weighted sum of the compressed array, and the
// permutations between mesh and cluster order.  (The plain all-frequency product runs on the
// matrix cores: mfma.hip.)
//
// y_l = A(s_l)^T x_l                                     (transposed product, per frequency)
// y   = sum_b sum_d H_{b,d} sum_l (I (x) f_{b,d}[l]) W_l  (eq. (3DacaMult))
//
// The transposed product walks column chunks of RCE elements: factored faces H = Ubar Vbar^H
// go through T' = Ubar^T X (k_far_products_t) and conj(Vbar) T'; the fibre acts on the output
// side.  The weighted sum contracts the fibres with W once per face and runs matrix-vector
// products bound by the HBM reads of the stored faces.  Arithmetic is FP64 (faces stored in
// complex64 are widened on load).
#include "aca3d.hpp"

namespace bem {

namespace {

constexpr int RCE = APPLY_ROW_CHUNK;  // elements per row chunk (48 rows)
constexpr int NC = 64;   // columns (rhs x frequency) per tile
constexpr int KR = 24;   // scalar columns of a face (8 elements) per staged tile of the row kernel
constexpr int KTF = 24;  // rows of Vbar per staged tile in the far products
constexpr int KMAXF = 96;  // largest rank of a factored face
constexpr int WGA = 256;

template <typename T> __device__ __forceinline__ zd ldz(const cx<T>* p) { return {(double)p->re, (double)p->im}; }

// z = f (3x3, row-major complex128) * v (3)
__device__ __forceinline__ void mul3(const zd* f, const zd* v, zd* z)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) z[a] = f[3 * a] * v[0] + f[3 * a + 1] * v[1] + f[3 * a + 2] * v[2];
}

// Fs[cl] = f[l] (3x3) of column c0 + cl (col = r L + l), or the selector fibre of a dense
// fallback face; read after a barrier.
__device__ __forceinline__ void stage_fibres(const ApplyArgs& A, const ApplyFace& F, int c0, int ncols, zd (*Fs)[9])
{
    const zd* fib = (const zd*)(A.pool + F.fib_off);
    for (int e = threadIdx.x; e < NC * 9; e += WGA) {
        const int cl = e / 9, t = e - 9 * (e / 9);
        const int col = c0 + cl, l = col % A.L;
        zd v = {0.0, 0.0};
        if (col < ncols) {
            if (F.sel) v = (l == F.ksel && (t == 0 || t == 4 || t == 8)) ? zd{1.0, 0.0} : zd{0.0, 0.0};
            else v = fib[(size_t)l * 9 + t];
        }
        Fs[cl][t] = v;
    }
}

// Y[rows][cols] += Hs[rows][k] Zs[k][cols] over one staged tile; thread = element row er
// (3 rows) x columns cq, cq + 16, cq + 32, cq + 48: 12 complex accumulators, 7 LDS reads
// per 12 complex multiply-adds.  Lanes of a wavefront read consecutive Zs entries and Hs rows
// are padded to an odd number of entries, so neither read has bank conflicts.
template <int KTL>
__device__ __forceinline__ void tile_mac(const zd (*Hs)[KTL], const zd (*Zs)[NC], int nk, int er, int cq, zd (*acc)[4])
{
    for (int k = 0; k < nk; ++k) {
        zd z[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) z[v] = Zs[k][cq + 16 * v];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const zd h = Hs[3 * er + a][k];
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[a][v] = fma_c(h, z[v], acc[a][v]);
        }
    }
}

// y rows of row chunk g = sum of its segments' partial rows, in segment order
template <bool WEIGHTED>
__global__ __launch_bounds__(256) void k_reduce_rows(ApplyArgs A, int ncols, zd* yout)
{
    const int g = blockIdx.x;
    const int rsz = A.row_size[g], rs0 = A.row_start[g];
    const int q = blockIdx.y * 256 + threadIdx.x;  // (row, col) with col fastest
    if (q >= 3 * rsz * ncols) return;
    const int row = q / ncols, col = q - row * ncols;
    zd s = {0.0, 0.0};
    for (int sg = A.group_seg[g]; sg < A.group_seg[g + 1]; ++sg) s += A.pbuf[((size_t)sg * 3 * RCE + row) * ncols + col];
    if (WEIGHTED) {
        yout[3 * (size_t)rs0 + row] = s;
    } else {
        const size_t M = 3 * (size_t)A.K;
        const int l = col % A.L, r = col / A.L;
        yout[((size_t)r * A.L + l) * M + 3 * (size_t)rs0 + row] = s;
    }
}

// ---------------------------------------------------------------- transposed products
// y_l = A(s_l)^T x_l: block (J, I) of the transpose is sum_d (I (x) f_d[l]^T) H_d^T, the fibre
// acting on the output side.  Factored faces: H^T = conj(Vbar) Ubar^T, so the far products
// form T' = Ubar^T X (plain rows of x, no fibre) and the row kernel multiplies conj(Vbar).

// T'[t][col] = sum_r Ubar[r][t] x[col][3 rb + r], r < 3m; thread = 3 ranks x 8 columns
template <typename T>
__device__ void far_products_face_t(const ApplyArgs& A, const ApplyFace& F, int ncols, int c0, zd (*Us)[KMAXF],
                                    zd (*Zs)[NC])
{
    const BlockIn B = A.blocks[F.block];
    const int m = B.rs, kk = F.kk;
    const cx<T>* U = (const cx<T>*)(A.pool + F.face_off);
    const int tr = threadIdx.x & 31, cg = threadIdx.x >> 5;
    const size_t M = 3 * (size_t)A.K;
    zd acc[3][8];
#pragma unroll
    for (int u = 0; u < 3; ++u)
#pragma unroll
        for (int v = 0; v < 8; ++v) acc[u][v] = {0.0, 0.0};
    for (int k0 = 0; k0 < 3 * m; k0 += KTF) {
        const int nk = min(KTF, 3 * m - k0);
        __syncthreads();
        for (int e = threadIdx.x; e < KTF * kk; e += WGA) {
            const int kr = e / kk, t = e - kr * kk;
            Us[kr][t] = kr < nk ? ldz(U + (size_t)(k0 + kr) * kk + t) : zd{0.0, 0.0};
        }
        for (int e = threadIdx.x; e < KTF * NC; e += WGA) {
            const int kr = e / NC, cl = e - kr * NC, col = c0 + cl;
            Zs[kr][cl] = (kr < nk && col < ncols) ? A.x[(size_t)col * M + 3 * (size_t)B.rb + k0 + kr] : zd{0.0, 0.0};
        }
        __syncthreads();
        for (int k = 0; k < nk; ++k) {
            zd uu[3];
#pragma unroll
            for (int u = 0; u < 3; ++u) uu[u] = tr + 32 * u < kk ? Us[k][tr + 32 * u] : zd{0.0, 0.0};
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const zd z = Zs[k][8 * cg + v];
#pragma unroll
                for (int u = 0; u < 3; ++u) acc[u][v] = fma_c(uu[u], z, acc[u][v]);
            }
        }
    }
    zd* Tout = A.tbuf + F.t_off * (size_t)ncols;
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        const int t = tr + 32 * u;
        if (t >= kk) continue;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int col = c0 + 8 * cg + v;
            if (col < ncols) Tout[(size_t)t * ncols + col] = acc[u][v];
        }
    }
}

__global__ __launch_bounds__(WGA) void k_far_products_t(ApplyArgs A, const int* far_list, int ncols)
{
    __shared__ zd Us[KTF][KMAXF];
    __shared__ zd Zs[KTF][NC];
    const ApplyFace F = A.faces[far_list[blockIdx.x]];
    const int c0 = blockIdx.y * NC;
    if (F.fp32) far_products_face_t<float>(A, F, ncols, c0, Us, Zs);
    else far_products_face_t<double>(A, F, ncols, c0, Us, Zs);
}

// Rows of the transpose: work item = (segment sg of a column chunk's faces, column tile).
// Per face the product H^T x (or conj(Vbar) T') is accumulated apart and the face's fibre,
// transposed, is applied per column before it joins the chunk's rows.
__global__ __launch_bounds__(WGA) void k_rows_t(ApplyArgs A, int ncols, int nitems)
{
    __shared__ zd Hs[3 * RCE][KR + 1];
    __shared__ zd Zs[KR][NC];
    __shared__ zd Fs[NC][9];
    const size_t M = 3 * (size_t)A.K;
    for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
        const int tile = w / A.nseg, sg = w - tile * A.nseg, c0 = tile * NC;
        const int g = A.seg_group[sg];
        const int er = threadIdx.x >> 4, cq = threadIdx.x & 15;
        const int cs0 = A.row_start[g], csz = A.row_size[g];
        zd acc[3][4];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[a][v] = {0.0, 0.0};
        for (int q = A.seg_begin[sg]; q < A.seg_begin[sg + 1]; ++q) {
            const ApplyFace F = A.faces[A.row_faces[q]];
            if (F.kk < 0) continue;
            const BlockIn B = A.blocks[F.block];
            const int m = B.rs, n = B.cs;
            const int joff = cs0 - B.cb;  // first column element of the chunk inside the block
            zd tmp[3][4];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int v = 0; v < 4; ++v) tmp[a][v] = {0.0, 0.0};
            __syncthreads();
            stage_fibres(A, F, c0, ncols, Fs);
            const int kin = F.kk == 0 ? 3 * m : F.kk;
            for (int k0 = 0; k0 < kin; k0 += KR) {
                const int nk = min(KR, kin - k0);
                __syncthreads();
                for (int e = threadIdx.x; e < 3 * RCE * KR; e += WGA) {
                    const int kc = e / (3 * RCE), r = e - kc * (3 * RCE);
                    zd h = {0.0, 0.0};
                    if (r < 3 * csz && kc < nk) {
                        if (F.kk == 0) {
                            const size_t o = (size_t)(k0 + kc) * (3 * (size_t)n) + 3 * joff + r;
                            h = F.fp32 ? ldz((const zf*)(A.pool + F.face_off) + o) : ((const zd*)(A.pool + F.face_off))[o];
                        } else {
                            const size_t o = (size_t)3 * m * F.kk + (size_t)(3 * joff + r) * F.kk + k0 + kc;
                            h = conj(F.fp32 ? ldz((const zf*)(A.pool + F.face_off) + o) : ((const zd*)(A.pool + F.face_off))[o]);
                        }
                    }
                    Hs[r][kc] = h;
                }
                for (int e = threadIdx.x; e < KR * NC; e += WGA) {
                    const int kr = e / NC, cl = e - kr * NC, col = c0 + cl;
                    zd z = {0.0, 0.0};
                    if (kr < nk && col < ncols)
                        z = F.kk == 0 ? A.x[(size_t)col * M + 3 * (size_t)B.rb + k0 + kr]
                                      : A.tbuf[(F.t_off + k0 + kr) * (size_t)ncols + col];
                    Zs[kr][cl] = z;
                }
                __syncthreads();
                tile_mac<KR + 1>(Hs, Zs, nk, er, cq, tmp);
            }
            // acc[a][v] += sum_b f[l_v][b][a] tmp[b][v]
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const zd* f = Fs[cq + 16 * v];
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) acc[a][v] = fma_c(f[3 * b + a], tmp[b][v], acc[a][v]);
            }
        }
        if (er < csz) {
            zd* pb = A.pbuf + (size_t)sg * 3 * RCE * ncols;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int col = c0 + cq + 16 * v;
                if (col >= ncols) continue;
#pragma unroll
                for (int a = 0; a < 3; ++a) pb[(size_t)(3 * er + a) * ncols + col] = acc[a][v];
            }
        }
    }
}

// One column (the weighted sum): the products are matrix-vector products bound by the HBM
// reads of the stored faces, so they run without the column tiles of the general kernels.

__device__ __forceinline__ zd wsum_z(zd v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        v.re += __shfl_xor(v.re, o, 64);
        v.im += __shfl_xor(v.im, o, 64);
    }
    return v;
}

// far faces: T[t] = sum_k conj(Vbar[k][t]) z[k] with z the face's contracted vector; one
// workgroup per face, waves over k, lanes over t (t and t + 64)
__global__ __launch_bounds__(256) void k_far_vec(ApplyArgs A, const int* far_list, const zd* zw_all)
{
    __shared__ zd part[4][KMAXF];
    const ApplyFace F = A.faces[far_list[blockIdx.x]];
    const BlockIn B = A.blocks[F.block];
    const int kk = F.kk, nk = 3 * B.cs, m = B.rs;
    const zd* z = zw_all + F.zw_off;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    zd a0 = {0.0, 0.0}, a1 = {0.0, 0.0};
    for (int k = wv; k < nk; k += 4) {
        const zd zk = z[k];
        const size_t o = (size_t)3 * m * kk + (size_t)k * kk;
        if (F.fp32) {
            const zf* V = (const zf*)(A.pool + F.face_off) + o;
            if (lane < kk) a0 = fma_c(conj(ldz(V + lane)), zk, a0);
            if (lane + 64 < kk) a1 = fma_c(conj(ldz(V + lane + 64)), zk, a1);
        } else {
            const zd* V = (const zd*)(A.pool + F.face_off) + o;
            if (lane < kk) a0 = fma_c(conj(V[lane]), zk, a0);
            if (lane + 64 < kk) a1 = fma_c(conj(V[lane + 64]), zk, a1);
        }
    }
    part[wv][lane] = a0;
    if (lane + 64 < KMAXF) part[wv][lane + 64] = a1;
    __syncthreads();
    if (threadIdx.x < kk) {
        zd sum = {0.0, 0.0};
        for (int w = 0; w < 4; ++w) sum += part[w][threadIdx.x];
        A.tbuf[F.t_off + threadIdx.x] = sum;
    }
}

// rows: segment sg of a row chunk; wave wv owns the rows wv, wv + 4, ... of the chunk's
// 3 rsz rows, lanes run along the face's columns (dense face: the contracted vector,
// factors: T); partial rows to pbuf, summed by k_reduce_rows
__global__ __launch_bounds__(256) void k_rows_vec(ApplyArgs A, const zd* zw_all)
{
    constexpr int RPW = 3 * RCE / 4;
    const int sg = blockIdx.x, g = A.seg_group[sg];
    const int rs0 = A.row_start[g], nrow = 3 * A.row_size[g];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    zd acc[RPW];
#pragma unroll
    for (int u = 0; u < RPW; ++u) acc[u] = {0.0, 0.0};
    for (int q = A.seg_begin[sg]; q < A.seg_begin[sg + 1]; ++q) {
        const ApplyFace F = A.faces[A.row_faces[q]];
        if (F.kk < 0) continue;
        const BlockIn B = A.blocks[F.block];
        const int ioff = rs0 - B.rb;
        const zd* z = F.kk == 0 ? zw_all + F.zw_off : A.tbuf + F.t_off;
        const int ncol = F.kk == 0 ? 3 * B.cs : F.kk;
        for (int c0 = 0; c0 < ncol; c0 += 64) {
            const int c = c0 + lane;
            if (c >= ncol) continue;
            const zd zc = z[c];
#pragma unroll
            for (int u = 0; u < RPW; ++u) {
                const int r = wv + 4 * u;
                if (r < nrow) {
                    const size_t o = (size_t)(3 * ioff + r) * ncol + c;
                    const zd h = F.fp32 ? ldz((const zf*)(A.pool + F.face_off) + o) : ((const zd*)(A.pool + F.face_off))[o];
                    acc[u] = fma_c(h, zc, acc[u]);
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < RPW; ++u) {
        const zd sv = wsum_z(acc[u]);
        const int r = wv + 4 * u;
        if (lane == 0 && r < nrow) A.pbuf[(size_t)sg * 3 * RCE + r] = sv;
    }
}

// zw[face][3j + c] = sum_l (f[l] W_l[J])_c  (the fibre contraction of eq. (3DacaMult)); one
// wavefront per face, four faces per workgroup, lanes over the block's column elements
__global__ __launch_bounds__(256) void k_contract(ApplyArgs A, const zd* W, zd* zw_all)
{
    const int fi = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (fi >= A.nfaces) return;
    const ApplyFace F = A.faces[fi];
    const BlockIn B = A.blocks[F.block];
    zd* zw = zw_all + F.zw_off;
    for (int j = lane; j < B.cs; j += 64) {
        zd s[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
        for (int l = 0; l < A.L; ++l) {
            if (F.sel && l != F.ksel) continue;
            const zd* w = W + (size_t)l * 3 * A.K + 3 * (size_t)(B.cb + j);
            zd v[3] = {w[0], w[1], w[2]}, z[3];
            if (F.sel) {
                z[0] = v[0];
                z[1] = v[1];
                z[2] = v[2];
            } else {
                mul3((const zd*)(A.pool + F.fib_off) + (size_t)l * 9, v, z);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) s[c] += z[c];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) zw[3 * (size_t)j + c] = s[c];
    }
}

// The same with one vector for every frequency (W_l = a x): zw = a (sum_l f[l]) x[J], the
// fibre sum taken once per face; one wavefront per face.
__global__ __launch_bounds__(256) void k_contract_sum(ApplyArgs A, const zd* x, double a, zd* zw_all)
{
    __shared__ zd Fb[4][9];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int fi = blockIdx.x * 4 + wv;
    const bool act = fi < A.nfaces;
    const ApplyFace F = A.faces[act ? fi : 0];
    if (lane < 9) {
        zd sum = {0.0, 0.0};
        if (act) {
            if (F.sel) {
                sum = (lane == 0 || lane == 4 || lane == 8) ? zd{1.0, 0.0} : zd{0.0, 0.0};
            } else {
                const zd* fib = (const zd*)(A.pool + F.fib_off);
                for (int l = 0; l < A.L; ++l) sum += fib[(size_t)l * 9 + lane];
            }
        }
        Fb[wv][lane] = sum * a;
    }
    __syncthreads();
    if (!act) return;
    const BlockIn B = A.blocks[F.block];
    zd* zw = zw_all + F.zw_off;
    for (int j = lane; j < B.cs; j += 64) {
        const zd* w = x + 3 * (size_t)(B.cb + j);
        const zd v[3] = {w[0], w[1], w[2]};
        zd z[3];
        mul3(Fb[wv], v, z);
#pragma unroll
        for (int c = 0; c < 3; ++c) zw[3 * (size_t)j + c] = z[c];
    }
}

__global__ __launch_bounds__(256) void k_permute(const zd* in, zd* out, const int* perm, int K, int L, int nrhs,
                                                 int64_t in_l_stride, int to_cluster)
{
    int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t total = (int64_t)nrhs * L * K;
    if (q >= total) return;
    int p = (int)(q % K);
    int l = (int)((q / K) % L);
    int r = (int)(q / ((int64_t)K * L));
    int e = perm[p];
    size_t M = 3 * (size_t)K;
    if (to_cluster) {
        const zd* src = in + (size_t)r * (in_l_stride ? L * (size_t)in_l_stride : M) + (size_t)l * in_l_stride + 3 * (size_t)e;
        zd* dst = out + ((size_t)r * L + l) * M + 3 * (size_t)p;
        dst[0] = src[0];
        dst[1] = src[1];
        dst[2] = src[2];
    } else {
        const zd* src = in + ((size_t)r * L + l) * M + 3 * (size_t)p;
        zd* dst = out + ((size_t)r * L + l) * M + 3 * (size_t)e;
        dst[0] = src[0];
        dst[1] = src[1];
        dst[2] = src[2];
    }
}

// Batched permutation between the mesh-order vectors of several operators and one
// cluster-order workspace [nrhs][L][3 Ktot] (operator o at element offset koff); blockIdx.y
// = operator.
__global__ __launch_bounds__(256) void k_permute_batch(BatchPermTable T, zd* work, int to_cluster)
{
    const BatchPerm& P = T.op[blockIdx.y];
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= (int64_t)T.nrhs * T.L * P.K) return;
    const int p = (int)(q % P.K);
    const int64_t rl = q / P.K;  // r L + l
    const int e = P.perm[p];
    zd* w = work + (size_t)rl * 3 * T.Ktot + 3 * (size_t)(P.koff + p);
    if (to_cluster) {
        const zd* src = P.x + (size_t)rl * 3 * P.K + 3 * (size_t)e;
        w[0] = src[0];
        w[1] = src[1];
        w[2] = src[2];
    } else {
        zd* dst = P.y + (size_t)rl * 3 * P.K + 3 * (size_t)e;
        dst[0] = w[0];
        dst[1] = w[1];
        dst[2] = w[2];
    }
}

}  // namespace

void launch_permute_batch(const BatchPermTable& T, int kmax, zd* work, bool to_cluster, hipStream_t st)
{
    if (T.nops < 1 || T.nops > MAX_BATCH_OPS) throw std::invalid_argument("batch of 1 to 16 operators");
    const int64_t total = (int64_t)T.nrhs * T.L * kmax;
    hipLaunchKernelGGL(k_permute_batch, dim3((unsigned)((total + 255) / 256), T.nops), dim3(256), 0, st, T, work,
                       (int)to_cluster);
    BEM_HIP_TRY(hipGetLastError());
}

void launch_permute(const zd* in, zd* out, const int* perm, int K, int L, int nrhs, int64_t in_l_stride, bool to_cluster,
                    hipStream_t st)
{
    int64_t total = (int64_t)nrhs * L * K;
    hipLaunchKernelGGL(k_permute, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, in, out, perm, K, L, nrhs,
                       in_l_stride, (int)to_cluster);
    BEM_HIP_TRY(hipGetLastError());
}

void launch_apply_t(const ApplyArgs& A, hipStream_t st)
{
    const int ncols = A.L * A.nrhs;
    const unsigned ct = (unsigned)((ncols + NC - 1) / NC);
    if (A.nfar > 0) hipLaunchKernelGGL(k_far_products_t, dim3(A.nfar, ct), dim3(WGA), 0, st, A, A.far_list, ncols);
    BEM_HIP_TRY(hipGetLastError());
    const long long items = (long long)A.nseg * ct;
    if (items >= (1LL << 31)) throw std::invalid_argument("too many row work items");
    hipLaunchKernelGGL(k_rows_t, dim3((unsigned)items), dim3(WGA), 0, st, A, ncols, (int)items);
    BEM_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL((k_reduce_rows<false>), dim3(A.nrow_groups, (3 * RCE * ncols + 255) / 256), dim3(256), 0, st, A,
                       ncols, A.y);
    BEM_HIP_TRY(hipGetLastError());
}

// W in cluster order [L][3K] (uniform: one vector [3K] used as a W for every l); zw:
// [nfaces][3K] workspace; y in cluster order [3K].
void launch_weighted(const ApplyArgs& A, const zd* W, zd* zw, zd* y, hipStream_t st, bool uniform, double scale)
{
    if (A.nfaces > 0) {
        if (uniform) hipLaunchKernelGGL(k_contract_sum, dim3((A.nfaces + 3) / 4), dim3(256), 0, st, A, W, scale, zw);
        else hipLaunchKernelGGL(k_contract, dim3((A.nfaces + 3) / 4), dim3(256), 0, st, A, W, zw);
        BEM_HIP_TRY(hipGetLastError());
    }
    if (A.nfar > 0) {
        hipLaunchKernelGGL(k_far_vec, dim3(A.nfar), dim3(256), 0, st, A, A.far_list, zw);
        BEM_HIP_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(k_rows_vec, dim3(A.nseg), dim3(256), 0, st, A, zw);
    BEM_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL((k_reduce_rows<true>), dim3(A.nrow_groups, (3 * RCE + 255) / 256), dim3(256), 0, st, A, 1, y);
    BEM_HIP_TRY(hipGetLastError());
}

}  // namespace bem
