// entries.hip -- raw entry generator, dense assembly of all frequency slices and dense
// all-frequency products (the uncompressed M x M x L array of Sec. 2.4).
#include "lib.hpp"

namespace bem {

template <bool MIXED>
__global__ __launch_bounds__(256) void k_entries(DevCtx c, int op, int64_t n, const int32_t* __restrict__ ii,
                                                 const int32_t* __restrict__ jj, const int32_t* __restrict__ ll,
                                                 zd* __restrict__ out)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    int i = ii[e], j = jj[e], l = ll[e];
    zd* o = out + e * 9;
    if (i < 0 || i >= c.geo.K || j < 0 || j >= c.geo.K || l < 0 || l >= c.fr.L) {
        for (int t = 0; t < 9; ++t) o[t] = {__builtin_nan(""), __builtin_nan("")};
        return;
    }
    blk b = entry_dispatch<MIXED>(c, op, i, j, l);
    for (int t = 0; t < 9; ++t) o[t] = b.a[t];
}

// ENTRY of the double layer weighted by the hat function of vertex op - OP_KL0 of element j
// (linear basis, FP64 rules)
__global__ __launch_bounds__(256) void k_entries_kl(DevCtx c, int op, int64_t n, const int32_t* __restrict__ ii,
                                                    const int32_t* __restrict__ jj, const int32_t* __restrict__ ll,
                                                    zd* __restrict__ out)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    int i = ii[e], j = jj[e], l = ll[e];
    zd* o = out + e * 9;
    if (i < 0 || i >= c.geo.K || j < 0 || j >= c.geo.K || l < 0 || l >= c.fr.L) {
        for (int t = 0; t < 9; ++t) o[t] = {__builtin_nan(""), __builtin_nan("")};
        return;
    }
    blk b[3];
    entry_kl3(c.geo, i, j, c.fr.s[l], c.fr.sinv[l], c.md, c.qt, b);
    const int v = op - OP_KL0;
    for (int t = 0; t < 9; ++t) o[t] = b[v].a[t];
}

void launch_entries(const DevCtx& c, int op, int mixed, int64_t n, const int32_t* i, const int32_t* j,
                    const int32_t* l, zd* out, hipStream_t st)
{
    if (n <= 0) return;
    dim3 grid((unsigned)((n + 255) / 256));
    if (op >= OP_KL0)
        hipLaunchKernelGGL(k_entries_kl, grid, dim3(256), 0, st, c, op, n, i, j, l, out);
    else if (mixed)
        hipLaunchKernelGGL(k_entries<true>, grid, dim3(256), 0, st, c, op, n, i, j, l, out);
    else
        hipLaunchKernelGGL(k_entries<false>, grid, dim3(256), 0, st, c, op, n, i, j, l, out);
    BEM_HIP_TRY(hipGetLastError());
}

// out[l][3i + a][3j + b] = ENTRY(i, j, l)[a][b]; thread per (j, i, l), 64 consecutive j per
// wavefront so that each row a of the 3x3 blocks is written as one contiguous segment.
template <bool MIXED>
__global__ __launch_bounds__(64) void k_dense_assemble(DevCtx c, int op, zd* __restrict__ out)
{
    const int K = c.geo.K;
    int j = blockIdx.x * 64 + threadIdx.x;
    int i = blockIdx.y;
    int l = blockIdx.z;
    if (j >= K) return;
    blk b = entry_dispatch<MIXED>(c, op, i, j, l);
    size_t M = (size_t)3 * K;
    zd* base = out + (size_t)l * M * M + (size_t)(3 * i) * M + 3 * j;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) base[(size_t)a * M + bb] = b.a[3 * a + bb];
}

void launch_dense_assemble(const DevCtx& c, int op, int mixed, zd* out, hipStream_t st)
{
    int K = c.geo.K;
    dim3 grid((K + 63) / 64, K, c.fr.L);
    if (mixed)
        hipLaunchKernelGGL(k_dense_assemble<true>, grid, dim3(64), 0, st, c, op, out);
    else
        hipLaunchKernelGGL(k_dense_assemble<false>, grid, dim3(64), 0, st, c, op, out);
    BEM_HIP_TRY(hipGetLastError());
}

__device__ __forceinline__ zd wave_sum(zd v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        v.re += __shfl_xor(v.re, o, 64);
        v.im += __shfl_xor(v.im, o, 64);
    }
    return v;
}

// y[r][l][row] = sum_col A[l][row][col] x[r][l][col]: one wavefront per (row, l, r),
// lanes stride over columns (coalesced rows of A).
__global__ __launch_bounds__(256) void k_dense_apply(const zd* __restrict__ A, int M, int L, int nrhs,
                                                     const zd* __restrict__ x, int64_t xls, zd* __restrict__ y)
{
    int lane = threadIdx.x & 63;
    int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    int64_t total = (int64_t)M * L * nrhs;
    if (w >= total) return;
    int row = (int)(w % M);
    int l = (int)((w / M) % L);
    int r = (int)(w / ((int64_t)M * L));
    const zd* a = A + ((size_t)l * M + row) * M;
    const zd* xv = x + (size_t)r * (xls ? (size_t)L * xls : (size_t)M) + (size_t)l * xls;
    zd acc = {0.0, 0.0};
    for (int col = lane; col < M; col += 64) acc = fma_c(a[col], xv[col], acc);
    acc = wave_sum(acc);
    if (lane == 0) y[((size_t)r * L + l) * M + row] = acc;
}

// y[r][l][c] = sum_row A[l][row][c] x[r][l][row] (the transpose): thread per (c, l, r), c
// fastest (coalesced along the rows of A)
__global__ __launch_bounds__(256) void k_dense_apply_t(const zd* __restrict__ A, int M, int L, int nrhs,
                                                       const zd* __restrict__ x, zd* __restrict__ y)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= (int64_t)M * L * nrhs) return;
    const int c = (int)(q % M);
    const int l = (int)((q / M) % L);
    const int r = (int)(q / ((int64_t)M * L));
    const zd* a = A + (size_t)l * M * M + c;
    const zd* xv = x + ((size_t)r * L + l) * M;
    zd acc = {0.0, 0.0};
    for (int row = 0; row < M; ++row) acc = fma_c(a[(size_t)row * M], xv[row], acc);
    y[((size_t)r * L + l) * M + c] = acc;
}

void launch_dense_apply_t(const zd* A, int M, int L, int nrhs, const zd* x, zd* y, hipStream_t st)
{
    const int64_t n = (int64_t)M * L * nrhs;
    hipLaunchKernelGGL(k_dense_apply_t, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, A, M, L, nrhs, x, y);
    BEM_HIP_TRY(hipGetLastError());
}

void launch_dense_apply(const zd* A, int M, int L, int nrhs, const zd* x, int64_t x_l_stride, zd* y,
                        hipStream_t st)
{
    int64_t waves = (int64_t)M * L * nrhs;
    dim3 grid((unsigned)((waves + 3) / 4));
    hipLaunchKernelGGL(k_dense_apply, grid, dim3(256), 0, st, A, M, L, nrhs, x, x_l_stride, y);
    BEM_HIP_TRY(hipGetLastError());
}

// y[row] = sum_l sum_col A[l][row][col] W[l][col]
__global__ __launch_bounds__(256) void k_dense_weighted(const zd* __restrict__ A, int M, int L,
                                                        const zd* __restrict__ W, zd* __restrict__ y)
{
    int lane = threadIdx.x & 63;
    int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= M) return;
    zd acc = {0.0, 0.0};
    for (int l = 0; l < L; ++l) {
        const zd* a = A + ((size_t)l * M + row) * M;
        const zd* wv = W + (size_t)l * M;
        for (int col = lane; col < M; col += 64) acc = fma_c(a[col], wv[col], acc);
    }
    acc = wave_sum(acc);
    if (lane == 0) y[row] = acc;
}

void launch_dense_weighted(const zd* A, int M, int L, const zd* W, zd* y, hipStream_t st)
{
    dim3 grid((M + 3) / 4);
    hipLaunchKernelGGL(k_dense_weighted, grid, dim3(256), 0, st, A, M, L, W, y);
    BEM_HIP_TRY(hipGetLastError());
}

}  // namespace bem
