// apply.hip -- all-frequency product of the compressed array and the gCQ weighted sum.
//
// y_l = sum_b sum_d H_{b,d} (I (x) f_{b,d}[l]) x_l      (per frequency l and right-hand side)
// y   = sum_b sum_d H_{b,d} sum_l (I (x) f_{b,d}[l]) W_l  (eq. (3DacaMult))
// Far faces H = Ubar Vbar^H are applied as Ubar (Vbar^H Z); near faces densely.  Rows are
// owned by one thread per (row, column) so the sums are formed in a fixed order (no atomics).
#include "aca3d.hpp"

namespace bem {

namespace {

constexpr int CW = 16;    // columns (frequency x rhs) per workgroup
constexpr int RCH = 16;   // elements per row chunk (48 rows)
constexpr int MAXN = 64;  // largest near-field column cluster staged at once (elements)

template <typename T> __device__ __forceinline__ zd ldz(const cx<T>* p) { return {(double)p->re, (double)p->im}; }

// z = f (3x3, row-major complex128) * v (3)
__device__ __forceinline__ void mul3(const zd* f, const zd* v, zd* z)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) z[a] = f[3 * a] * v[0] + f[3 * a + 1] * v[1] + f[3 * a + 2] * v[2];
}

// Z[3j + c][col] for a face: col = (l, r) -> (f[l] x_r,l[J])_c, or the contracted vector.
template <bool WEIGHTED>
__device__ __forceinline__ void z_entry(const ApplyArgs& A, const ApplyFace& F, const BlockIn& B, const zd* zw, int j,
                                        int col, zd* z)
{
    if (WEIGHTED) {
        const zd* v = zw + 3 * (size_t)j;
        z[0] = v[0];
        z[1] = v[1];
        z[2] = v[2];
        return;
    }
    int L = A.L;
    int l = col % L, r = col / L;
    const zd* xv = A.x + ((size_t)r * L + l) * 3 * A.K + 3 * (size_t)(B.cb + j);
    if (F.sel) {
        if (l == F.ksel) {
            z[0] = xv[0];
            z[1] = xv[1];
            z[2] = xv[2];
        } else {
            z[0] = z[1] = z[2] = {0.0, 0.0};
        }
        return;
    }
    const zd* f = (const zd*)(A.pool + F.fib_off) + (size_t)l * 9;
    zd v[3] = {xv[0], xv[1], xv[2]};
    mul3(f, v, z);
}

// far faces: T[t][col] = sum_{j, c} conj(Vbar[3j + c, t]) Z[3j + c][col]   (Vbar row-major)
template <typename T, bool WEIGHTED>
__device__ void far_products_face(const ApplyArgs& A, const ApplyFace& F, const zd* zw_all, int ncols)
{
    const BlockIn B = A.blocks[F.block];
    const int m = B.rs, n = B.cs, kk = F.kk;
    const cx<T>* V = (const cx<T>*)(A.pool + F.face_off) + (size_t)3 * m * kk;
    const zd* zw = WEIGHTED ? zw_all + F.zw_off : nullptr;
    zd* Tout = A.tbuf + F.t_off * (size_t)ncols;
    for (int q = threadIdx.x; q < kk * ncols; q += 256) {
        int col = q / kk, t = q - col * kk;  // consecutive threads: consecutive t (contiguous Vbar rows)
        zd acc = {0.0, 0.0};
        for (int j = 0; j < n; ++j) {
            zd z[3];
            z_entry<WEIGHTED>(A, F, B, zw, j, col, z);
#pragma unroll
            for (int c = 0; c < 3; ++c) acc += conj_mul(ldz(V + (size_t)(3 * j + c) * kk + t), z[c]);
        }
        Tout[(size_t)t * ncols + col] = acc;
    }
}

template <bool WEIGHTED>
__global__ __launch_bounds__(256) void k_far_products(ApplyArgs A, const zd* zw_all, int ncols)
{
    const ApplyFace F = A.faces[blockIdx.x];
    if (F.kk <= 0) return;
    if (F.fp32) far_products_face<float, WEIGHTED>(A, F, zw_all, ncols);
    else far_products_face<double, WEIGHTED>(A, F, zw_all, ncols);
}

// rows: one workgroup per (row chunk, column chunk); thread = (row slot, column)
template <bool WEIGHTED>
__global__ __launch_bounds__(256) void k_rows(ApplyArgs A, const zd* zw_all, int ncols, zd* yout)
{
    __shared__ zd Zs[3 * MAXN * CW];
    const int g = blockIdx.x;
    const int c0 = blockIdx.y * CW;
    const int col_l = threadIdx.x % CW, slot = threadIdx.x / CW;  // 16 slots x 16 columns
    const int col = c0 + col_l;
    const int rs0 = A.row_start[g], rsz = A.row_size[g];
    zd acc[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    // each slot owns element row (rs0 + slot) if slot < rsz: 3 rows a = 0..2
    for (int q = A.row_ptr[g]; q < A.row_ptr[g + 1]; ++q) {
        const int fi = A.row_faces[q];
        const ApplyFace F = A.faces[fi];
        if (F.kk < 0) continue;
        const BlockIn B = A.blocks[F.block];
        const int m = B.rs, n = B.cs;
        const int ioff = rs0 - B.rb;  // first element row of the chunk inside the block
        const zd* zw = WEIGHTED ? zw_all + F.zw_off : nullptr;
        if (F.kk == 0) {
            const zd* H = (const zd*)(A.pool + F.face_off);
            const zf* Hf = (const zf*)(A.pool + F.face_off);
            const size_t ld = 3 * (size_t)n;
            for (int j0 = 0; j0 < n; j0 += MAXN) {
                int nj = min(MAXN, n - j0);
                __syncthreads();
                for (int e = threadIdx.x; e < nj * CW; e += 256) {
                    int jj = e / CW, cl = e - jj * CW;
                    zd z[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
                    if (c0 + cl < ncols) z_entry<WEIGHTED>(A, F, B, zw, j0 + jj, c0 + cl, z);
#pragma unroll
                    for (int c = 0; c < 3; ++c) Zs[(3 * jj + c) * CW + cl] = z[c];
                }
                __syncthreads();
                if (slot < rsz) {
                    const size_t o0 = (size_t)(3 * (ioff + slot)) * ld + 3 * j0;
                    if (F.fp32) {
                        for (int jc = 0; jc < 3 * nj; ++jc) {
                            zd z = Zs[jc * CW + col_l];
#pragma unroll
                            for (int a = 0; a < 3; ++a) acc[a] = fma_c(ldz(Hf + o0 + (size_t)a * ld + jc), z, acc[a]);
                        }
                    } else {
                        for (int jc = 0; jc < 3 * nj; ++jc) {
                            zd z = Zs[jc * CW + col_l];
#pragma unroll
                            for (int a = 0; a < 3; ++a) acc[a] = fma_c(H[o0 + (size_t)a * ld + jc], z, acc[a]);
                        }
                    }
                }
            }
        } else if (slot < rsz && col < ncols) {
            const int kk = F.kk;
            const zd* Tf = A.tbuf + F.t_off * (size_t)ncols;
            const size_t r0 = (size_t)(3 * (ioff + slot)) * kk;
            if (F.fp32) {
                const zf* U = (const zf*)(A.pool + F.face_off) + r0;
                for (int t = 0; t < kk; ++t) {
                    zd tv = Tf[(size_t)t * ncols + col];
#pragma unroll
                    for (int a = 0; a < 3; ++a) acc[a] = fma_c(ldz(U + (size_t)a * kk + t), tv, acc[a]);
                }
            } else {
                const zd* U = (const zd*)(A.pool + F.face_off) + r0;
                for (int t = 0; t < kk; ++t) {
                    zd tv = Tf[(size_t)t * ncols + col];
#pragma unroll
                    for (int a = 0; a < 3; ++a) acc[a] = fma_c(U[(size_t)a * kk + t], tv, acc[a]);
                }
            }
        }
        (void)m;
    }
    if (slot < rsz && col < ncols) {
        size_t M = 3 * (size_t)A.K;
        if (WEIGHTED) {
#pragma unroll
            for (int a = 0; a < 3; ++a) yout[3 * (size_t)(rs0 + slot) + a] = acc[a];
        } else {
            int l = col % A.L, r = col / A.L;
#pragma unroll
            for (int a = 0; a < 3; ++a) yout[((size_t)r * A.L + l) * M + 3 * (size_t)(rs0 + slot) + a] = acc[a];
        }
    }
}

// zw[face][3j + c] = sum_l (f[l] W_l[J])_c  (the fibre contraction of eq. (3DacaMult))
__global__ __launch_bounds__(256) void k_contract(ApplyArgs A, const zd* W, zd* zw_all)
{
    int fi = blockIdx.x;
    const ApplyFace F = A.faces[fi];
    const BlockIn B = A.blocks[F.block];
    zd* zw = zw_all + F.zw_off;
    for (int j = threadIdx.x; j < B.cs; j += 256) {
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

}  // namespace

void launch_permute(const zd* in, zd* out, const int* perm, int K, int L, int nrhs, int64_t in_l_stride, bool to_cluster,
                    hipStream_t st)
{
    int64_t total = (int64_t)nrhs * L * K;
    hipLaunchKernelGGL(k_permute, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, in, out, perm, K, L, nrhs,
                       in_l_stride, (int)to_cluster);
    BEM_HIP_TRY(hipGetLastError());
}

void launch_apply(const ApplyArgs& A, hipStream_t st)
{
    int ncols = A.L * A.nrhs;
    if (A.nfaces > 0) hipLaunchKernelGGL((k_far_products<false>), dim3(A.nfaces), dim3(256), 0, st, A, nullptr, ncols);
    BEM_HIP_TRY(hipGetLastError());
    dim3 grid(A.nrow_groups, (ncols + CW - 1) / CW);
    hipLaunchKernelGGL((k_rows<false>), grid, dim3(256), 0, st, A, nullptr, ncols, A.y);
    BEM_HIP_TRY(hipGetLastError());
}

// W in cluster order [L][3K]; zw: [nfaces][3K] workspace; y in cluster order [3K].
void launch_weighted(const ApplyArgs& A, const zd* W, zd* zw, zd* y, hipStream_t st)
{
    if (A.nfaces > 0) {
        hipLaunchKernelGGL(k_contract, dim3(A.nfaces), dim3(256), 0, st, A, W, zw);
        BEM_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL((k_far_products<true>), dim3(A.nfaces), dim3(256), 0, st, A, zw, 1);
        BEM_HIP_TRY(hipGetLastError());
    }
    dim3 grid(A.nrow_groups, 1);
    hipLaunchKernelGGL((k_rows<true>), grid, dim3(256), 0, st, A, zw, 1, y);
    BEM_HIP_TRY(hipGetLastError());
}

}  // namespace bem
