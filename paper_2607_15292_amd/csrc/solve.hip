// solve.hip -- vector kernels of the batched GMRES solve: every column (right-hand side x
// frequency) is an independent complex system of size N = 3K; vectors are stored [ncols][N]
// like the products' inputs, Krylov bases as consecutive such arrays.
#include "solve.hpp"

namespace bem {

namespace {

constexpr int WS = 256;

__device__ __forceinline__ double wsum_s(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// out[i][c] = <V_i[c], w[c]> = sum_n conj(V_i[c][n]) w[c][n] (one workgroup per (c, i),
// fixed-order reduction)
__global__ __launch_bounds__(WS) void k_dots(const zd* V, size_t vstride, const zd* w, int N, int ncols, zd* out)
{
    __shared__ double red[2][WS / 64];
    const int c = blockIdx.x, i = blockIdx.y;
    const zd* a = V + (size_t)i * vstride + (size_t)c * N;
    const zd* b = w + (size_t)c * N;
    double re = 0.0, im = 0.0;
    for (int n = threadIdx.x; n < N; n += WS) {
        const zd t = conj_mul(a[n], b[n]);
        re += t.re;
        im += t.im;
    }
    re = wsum_s(re);
    im = wsum_s(im);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wv] = re;
        red[1][wv] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sr = 0.0, si = 0.0;
        for (int t = 0; t < WS / 64; ++t) {
            sr += red[0][t];
            si += red[1][t];
        }
        out[(size_t)i * ncols + c] = {sr, si};
    }
}

// w[c][n] += sign sum_{i < nvec} h[i][c] V_i[c][n]
__global__ __launch_bounds__(WS) void k_combine(zd* w, const zd* V, size_t vstride, const zd* h, int nvec, int N,
                                                int ncols, double sign)
{
    const size_t q = (size_t)blockIdx.x * WS + threadIdx.x;
    if (q >= (size_t)N * ncols) return;
    const int c = (int)(q / N);
    zd s = {0.0, 0.0};
    for (int i = 0; i < nvec; ++i) s = fma_c(h[(size_t)i * ncols + c], V[(size_t)i * vstride + q], s);
    w[q] += s * sign;
}

// dst[c][n] = src[c][n] * scale[c]
__global__ __launch_bounds__(WS) void k_scale_cols(zd* dst, const zd* src, const double* scale, int N, int ncols)
{
    const size_t q = (size_t)blockIdx.x * WS + threadIdx.x;
    if (q >= (size_t)N * ncols) return;
    dst[q] = src[q] * scale[q / N];
}

// z = a x + b y (complex128 arrays of n entries; real a, b)
__global__ __launch_bounds__(WS) void k_axpby(zd* z, double a, const zd* x, double b, const zd* y, size_t n)
{
    const size_t q = (size_t)blockIdx.x * WS + threadIdx.x;
    if (q >= n) return;
    z[q] = x[q] * a + y[q] * b;
}

// out[l][m] = (W ? W[l][m] : 0) + a v[m] for l < L
__global__ __launch_bounds__(WS) void k_cq_fill(zd* out, const zd* W, const zd* v, double a, int L, int M)
{
    const size_t q = (size_t)blockIdx.x * WS + threadIdx.x;
    if (q >= (size_t)L * M) return;
    const zd t = v[q % M] * a;
    out[q] = W ? W[q] + t : t;
}

// W[l][m] = zinv[l] (W[l][m] + a v[m]): one step of the history recurrence
__global__ __launch_bounds__(WS) void k_cq_update(zd* W, const zd* v, const zd* zinv, double a, int L, int M)
{
    const size_t q = (size_t)blockIdx.x * WS + threadIdx.x;
    if (q >= (size_t)L * M) return;
    W[q] = zinv[q / M] * (W[q] + v[q % M] * a);
}

inline unsigned blocks_for(size_t n) { return (unsigned)((n + WS - 1) / WS); }

}  // namespace

void launch_cq_fill(zd* out, const zd* W, const zd* v, double a, int L, int M, hipStream_t st)
{
    hipLaunchKernelGGL(k_cq_fill, dim3(blocks_for((size_t)L * M)), dim3(WS), 0, st, out, W, v, a, L, M);
    BEM_HIP_TRY(hipGetLastError());
}

void launch_cq_update(zd* W, const zd* v, const zd* zinv, double a, int L, int M, hipStream_t st)
{
    hipLaunchKernelGGL(k_cq_update, dim3(blocks_for((size_t)L * M)), dim3(WS), 0, st, W, v, zinv, a, L, M);
    BEM_HIP_TRY(hipGetLastError());
}

void launch_dots(const zd* V, size_t vstride, int nvec, const zd* w, int N, int ncols, zd* out, hipStream_t st)
{
    if (nvec <= 0 || ncols <= 0) return;
    hipLaunchKernelGGL(k_dots, dim3(ncols, nvec), dim3(WS), 0, st, V, vstride, w, N, ncols, out);
    BEM_HIP_TRY(hipGetLastError());
}

void launch_combine(zd* w, const zd* V, size_t vstride, const zd* h, int nvec, int N, int ncols, double sign,
                    hipStream_t st)
{
    if (nvec <= 0 || ncols <= 0) return;
    hipLaunchKernelGGL(k_combine, dim3(blocks_for((size_t)N * ncols)), dim3(WS), 0, st, w, V, vstride, h, nvec, N, ncols,
                       sign);
    BEM_HIP_TRY(hipGetLastError());
}

void launch_scale_cols(zd* dst, const zd* src, const double* scale, int N, int ncols, hipStream_t st)
{
    if (ncols <= 0) return;
    hipLaunchKernelGGL(k_scale_cols, dim3(blocks_for((size_t)N * ncols)), dim3(WS), 0, st, dst, src, scale, N, ncols);
    BEM_HIP_TRY(hipGetLastError());
}

void launch_axpby(zd* z, double a, const zd* x, double b, const zd* y, size_t n, hipStream_t st)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_axpby, dim3(blocks_for(n)), dim3(WS), 0, st, z, a, x, b, y, n);
    BEM_HIP_TRY(hipGetLastError());
}

}  // namespace bem
