// mfma.hip -- the all-frequency product of the compressed array on the matrix cores.
//
// y_l = sum_b sum_d H_{b,d} (I (x) f_{b,d}[l]) x_l for every frequency l and right-hand side
// (the face-fibre form of eq. (3DacaMult)).  Per face and tile of 64 columns col = (rhs, l)
// the work is a complex GEMM: Y[I, :] += H Z with Z[3j + c][col] = (f[l] x_{r,l}[J])_c, or,
// for factors H = Ubar Vbar^H, T = Vbar^H Z (k_far_mfma) followed by Y[I, :] += Ubar T.
//
// Complex products run as real MFMA products.  A complex matrix stored interleaved (re, im)
// is a real matrix A_r with twice the columns; with
//     B'[2k][2c] = Re Z[k][c],  B'[2k+1][2c] = -Im Z[k][c],
//     B'[2k][2c+1] = Im Z[k][c], B'[2k+1][2c+1] = Re Z[k][c]
// the real product A_r B' is Y interleaved (4 real multiply-adds per complex one).  Faces
// stored in complex64 (far field, mixed precision) use v_mfma_f32_16x16x4f32 with FP32
// accumulation; complex128 faces use v_mfma_f64_16x16x4f64.
//
// A workgroup of 8 wavefronts owns one row chunk (a piece of a leaf cluster of at most 42
// elements, 126 rows) and one column tile (64 complex = 128 real columns) and walks one
// segment of the chunk's faces of one precision.  Operand tiles of KC real k are staged in LDS with k
// contiguous: each lane reads VEC consecutive k values with one 16-byte load and feeds VEC
// MFMAs (the order of k inside a tile is a permutation shared by both operands).  Wave w
// owns the row tiles (w & 3) + 4u, u < 2, and the column tiles 4 (w >> 2) + v, v < 4.  Partial rows of the
// segments go to a workspace and are added in segment order (no atomics).
#include "aca3d.hpp"

namespace bem {

namespace {

constexpr int WGM = 512;                      // 8 wavefronts
constexpr int MTM = 3 * MFMA_ROW_CHUNK;       // rows of a chunk (126), the stride of the partial rows
constexpr int MTR = 128;                      // staged rows: 8 row tiles of 16
constexpr int MCOL = MFMA_COLS;               // complex columns of a tile (64)
constexpr int NTR = 2 * MFMA_COLS;            // real columns of a tile (128)

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename R> struct MM;
template <> struct MM<float> {
    using acc_t = f32x4;   // 4 outputs per lane
    using vec_t = f32x4;   // 4 consecutive k of one operand (16 bytes)
    static constexpr int VEC = 4;
    static constexpr int KC = 48;  // real k per staged tile
    __device__ static __forceinline__ acc_t mac(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // output row (inside the 16 x 16 tile) of register v of a lane; the column is lane & 15
    __device__ static __forceinline__ int orow(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct MM<double> {
    using acc_t = f64x4;
    using vec_t = f64x2;
    static constexpr int VEC = 2;
    static constexpr int KC = 24;
    __device__ static __forceinline__ acc_t mac(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int orow(int lane, int v) { return (lane >> 4) + 4 * v; }
};

template <typename R> constexpr int ldk() { return MM<R>::KC + 16 / (int)sizeof(R); }  // padded row

// Fs[cc] = f[l] (3x3) of column c0 + cc (col = r L + l), or the selector fibre of a dense
// fallback face
__device__ __forceinline__ void stage_fibres_m(const MApplyArgs& A, const ApplyFace& F, int c0, int ncols, zd (*Fs)[9])
{
    const zd* fib = (const zd*)(A.pool + F.fib_off);
    for (int e = threadIdx.x; e < MCOL * 9; e += WGM) {
        const int cc = e / 9, t = e - 9 * cc;
        const int col = c0 + cc, l = col % A.L;
        zd v = {0.0, 0.0};
        if (col < ncols) {
            if (F.sel) v = (l == F.ksel && (t == 0 || t == 4 || t == 8)) ? zd{1.0, 0.0} : zd{0.0, 0.0};
            else v = fib[(size_t)l * 9 + t];
        }
        Fs[cc][t] = v;
    }
}

// Bs: B' of the complex operand rows k0/2 .. k0/2 + KC/2 and the tile's 64 columns.
// Dense face: Z[kg][col] = (f[l] x_{r,l}[cb + kg / 3])_{kg % 3}; factors: T[kg][col].
template <typename R>
__device__ __forceinline__ void stage_b(const MApplyArgs& A, const BlockIn& B, const ApplyFace& F, bool dense, int k0,
                                        int nk, int c0, int ncols, const zd (*Fs)[9], R* Bs)
{
    constexpr int KC = MM<R>::KC, LD = ldk<R>();
    for (int e = threadIdx.x; e < (KC / 2) * MCOL; e += WGM) {
        const int cc = e / (KC / 2), kc = e - cc * (KC / 2);
        const int col = c0 + cc, kg = (k0 >> 1) + kc;
        zd z = {0.0, 0.0};
        if (2 * kc < nk && col < ncols) {
            if (dense) {
                const int j = kg / 3, a = kg - 3 * j;
                const int l = col % A.L, r = col / A.L;
                const zd* xv = A.x + ((size_t)r * A.L + l) * 3 * A.K + 3 * (size_t)(B.cb + j);
                z = fma_c(Fs[cc][3 * a + 2], xv[2], fma_c(Fs[cc][3 * a + 1], xv[1], Fs[cc][3 * a] * xv[0]));
            } else {
                z = A.tbuf[(F.t_off + kg) * (size_t)ncols + col];
            }
        }
        R* b0 = Bs + (2 * cc) * LD + 2 * kc;
        R* b1 = b0 + LD;
        b0[0] = (R)z.re;
        b0[1] = (R)-z.im;
        b1[0] = (R)z.im;
        b1[1] = (R)z.re;
    }
}

// acc[u][v] += As(row tile rt0 + 4u) Bs(column tile ct0 + v) over one staged tile
template <typename R, int NU>
__device__ __forceinline__ void mfma_tile(const R* As, const R* Bs, int rt0, int ct0, int nrt, int lane,
                                          typename MM<R>::acc_t (*acc)[4])
{
    using C = MM<R>;
    using vec_t = typename C::vec_t;
    constexpr int KC = C::KC, VEC = C::VEC, LD = ldk<R>();
    const int li = lane & 15, lg = lane >> 4;
#pragma unroll
    for (int s = 0; s < KC; s += 4 * VEC) {
        vec_t a[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int rt = rt0 + 4 * u;
            a[u] = rt < nrt ? *(const vec_t*)(As + (16 * rt + li) * LD + s + VEC * lg) : vec_t{};
        }
        // one B fragment live at a time keeps the FP64 variant within 128 registers
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const vec_t b = *(const vec_t*)(Bs + (16 * (ct0 + v) + li) * LD + s + VEC * lg);
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                if (rt0 + 4 * u >= nrt) continue;  // uniform over the wavefront
#pragma unroll
                for (int t = 0; t < VEC; ++t) acc[u][v] = C::mac(a[u][t], b[t], acc[u][v]);
            }
        }
    }
}

// Far faces: T[t][col] = sum_k conj(Vbar[k][t]) Z[k][col] for t < kk (<= 96), one workgroup per
// (face, column tile).  A = Vbar^H is staged as As[t][2k] = Re Vbar[k][t], As[t][2k+1] =
// -Im Vbar[k][t].
template <typename R>
__global__ __launch_bounds__(WGM, 4) void k_far_mfma(MApplyArgs A, int ncols, const int* list, int n)
{
    using C = MM<R>;
    constexpr int KC = C::KC, LD = ldk<R>();
    __shared__ __align__(16) R As[96 * LD];
    __shared__ __align__(16) R Bs[NTR * LD];
    __shared__ zd Fs[MCOL][9];
    const ApplyFace F = A.faces[list[blockIdx.x % n]];
    const int c0 = (blockIdx.x / n) * MCOL;
    const BlockIn B = A.blocks[F.block];
    const int kk = F.kk, nrt = (kk + 15) >> 4;
    const cx<R>* V = (const cx<R>*)(A.pool + F.face_off) + (size_t)3 * B.rs * kk;
    const int kreal = 6 * B.cs;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int rt0 = wv & 3, ct0 = 4 * (wv >> 2);
    typename C::acc_t acc[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = typename C::acc_t{};
    stage_fibres_m(A, F, c0, ncols, Fs);
    for (int k0 = 0; k0 < kreal; k0 += KC) {
        const int nk = min(KC, kreal - k0);
        __syncthreads();
        const int tr = 16 * nrt;
        for (int e = tid; e < tr * (KC / 2); e += WGM) {
            const int kc = e / tr, t = e - kc * tr;
            cx<R> v = {(R)0, (R)0};
            if (t < kk && 2 * kc < nk) v = V[(size_t)((k0 >> 1) + kc) * kk + t];
            As[t * LD + 2 * kc] = v.re;
            As[t * LD + 2 * kc + 1] = -v.im;
        }
        stage_b<R>(A, B, F, true, k0, nk, c0, ncols, Fs, Bs);
        __syncthreads();
        mfma_tile<R, 2>(As, Bs, rt0, ct0, nrt, lane, acc);
    }
    zd* Tout = A.tbuf + F.t_off * (size_t)ncols;
    const int li = lane & 15;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int rt = rt0 + 4 * u;
        if (rt >= nrt) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rc = 16 * (ct0 + v) + li, col = c0 + (rc >> 1);
            if (col >= ncols) continue;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const int t = 16 * rt + C::orow(lane, w);
                if (t < kk) ((double*)(Tout + (size_t)t * ncols + col))[rc & 1] = (double)acc[u][v][w];
            }
        }
    }
}

// Rows: one workgroup per (segment of one precision, column tile); the segment's partial rows
// go to pbuf[sg] and k_reduce_mrows adds them.  The segment is a sequence of jobs (face, tile of
// KC real k): the face rows of the chunk (A) and the input side (B') of a job are staged in
// one of two LDS buffers.  While the MFMAs of job j read one buffer, the global loads of job
// j + 1 are in flight in registers; after the MFMAs they are written to the other buffer (the
// fibre contraction Z = f x happens then), and one barrier ends the step.
struct RowJob {
    int q, k0;         // entry of row_faces, first real k of the tile
    int dense, kreal;  // dense face (else factors), real entries per face row
    long long face_off, fib_off, t_off;
    int kk, sel, ksel, rb, cb;
};

__device__ __forceinline__ void job_face(const MApplyArgs& A, int q, RowJob& J)
{
    const ApplyFace& F = A.faces[A.row_faces[q]];
    const BlockIn& B = A.blocks[F.block];
    J.q = q;
    J.k0 = 0;
    J.face_off = F.face_off;
    J.fib_off = F.fib_off;
    J.t_off = F.t_off;
    J.kk = F.kk;
    J.sel = F.sel;
    J.ksel = F.ksel;
    J.rb = B.rb;
    J.cb = B.cb;
    J.dense = F.kk == 0;
    J.kreal = J.dense ? 6 * B.cs : 2 * F.kk;
}

template <typename R>
__device__ __forceinline__ void put_b(R* bs, int zcc, int kc, zd z)
{
    constexpr int LD = ldk<R>();
    R* b0 = bs + (2 * zcc) * LD + 2 * kc;
    b0[0] = (R)z.re;
    b0[1] = (R)-z.im;
    b0[LD] = (R)z.im;
    b0[LD + 1] = (R)z.re;
}

// Staging of one job, written out in the kernel body (the loaded values must stay in
// registers across the MFMAs of the previous job; helper functions taking them by reference
// left them in memory).
// ROW_FETCH(J): global loads of job J into av[] (face entries) and x0..x2 (the three inputs
// of this thread's (column, element) pair: x of the element, or rows of T for factors).
#define ROW_FETCH(J)                                                                                    \
    do {                                                                                                \
        const int nk_ = min(KC, (J).kreal - (J).k0);                                                    \
        const R* H_ = (const R*)(A.pool + (J).face_off) + (size_t)3 * (rs0 - (J).rb) * (J).kreal + (J).k0; \
        _Pragma("unroll") for (int i = 0; i < APT; ++i)                                                 \
        {                                                                                               \
            const int e = tid + WGM * i, r = e / KC, kr = e - r * KC;                                   \
            av[i] = (r < nrows && kr < nk_) ? H_[(size_t)r * (J).kreal + kr] : (R)0;                    \
        }                                                                                               \
        const int kg0_ = ((J).k0 >> 1) + 3 * zjj;                                                       \
        x0 = x1 = x2 = zd{0.0, 0.0};                                                                    \
        if (zact && 6 * zjj < nk_) {                                                                    \
            if ((J).dense) {                                                                            \
                const zd* xv_ = A.x + ((size_t)zr * A.L + zl) * 3 * A.K + 3 * (size_t)((J).cb + kg0_ / 3); \
                x0 = xv_[0];                                                                            \
                x1 = xv_[1];                                                                            \
                x2 = xv_[2];                                                                            \
            } else {                                                                                    \
                const zd* tv_ = A.tbuf + ((J).t_off + kg0_) * (size_t)ncols + zcol;                   \
                x0 = tv_[0];                                                                            \
                if (kg0_ + 1 < (J).kk) x1 = tv_[ncols];                                               \
                if (kg0_ + 2 < (J).kk) x2 = tv_[2 * (size_t)ncols];                                   \
            }                                                                                           \
        }                                                                                               \
    } while (0)

// ROW_STORE(J, t): the registers of job J into LDS buffer t, with the fibre contraction
// Z = f[l] x for a dense face
#define ROW_STORE(J, t)                                                                                 \
    do {                                                                                                \
        R* as_ = As[t];                                                                                 \
        _Pragma("unroll") for (int i = 0; i < APT; ++i)                                                 \
        {                                                                                               \
            const int e = tid + WGM * i, r = e / KC, kr = e - r * KC;                                   \
            as_[r * LD + kr] = av[i];                                                                   \
        }                                                                                               \
        if (zcc < MCOL) {                                                                               \
            zd z0 = x0, z1 = x1, z2 = x2;                                                               \
            if ((J).dense && zact) {                                                                    \
                if ((J).sel) {                                                                        \
                    if (zl != (J).ksel) z0 = z1 = z2 = zd{0.0, 0.0};                                  \
                } else {                                                                                \
                    const zd* f = (const zd*)(A.pool + (J).fib_off) + (size_t)zl * 9;                 \
                    z0 = fma_c(f[2], x2, fma_c(f[1], x1, f[0] * x0));                                   \
                    z1 = fma_c(f[5], x2, fma_c(f[4], x1, f[3] * x0));                                   \
                    z2 = fma_c(f[8], x2, fma_c(f[7], x1, f[6] * x0));                                   \
                }                                                                                       \
            }                                                                                           \
            put_b<R>(Bs[t], zcc, 3 * zjj, z0);                                                          \
            put_b<R>(Bs[t], zcc, 3 * zjj + 1, z1);                                                      \
            put_b<R>(Bs[t], zcc, 3 * zjj + 2, z2);                                                      \
        }                                                                                               \
    } while (0)

template <typename R>
__global__ __launch_bounds__(WGM, 2) void k_rows_mfma(MApplyArgs A, int ncols, const int* seglist, int nsegs)
{
    using C = MM<R>;
    constexpr int KC = C::KC, LD = ldk<R>();
    constexpr int APT = MTR * KC / WGM;   // face entries staged per thread and job
    constexpr int EPT = KC / 6;           // column elements per job (KC real k = KC / 6 elements)
    static_assert(KC % 6 == 0 && (MTR * KC) % WGM == 0, "tile shape");
    __shared__ __align__(16) R As[2][MTR * LD];
    __shared__ __align__(16) R Bs[2][NTR * LD];
    const int sg = seglist[blockIdx.x % nsegs];
    const int c0 = (blockIdx.x / nsegs) * MCOL;
    const int g = A.seg_group[sg];
    const int rs0 = A.row_start[g], nrows = 3 * A.row_size[g];
    const int nrt = (nrows + 15) >> 4;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int rt0 = wv & 3, ct0 = 4 * (wv >> 2);
    // this thread's (column, element) pair of the input side of a job
    const int zcc = tid / EPT, zjj = tid - zcc * EPT;
    const int zcol = c0 + zcc;
    const bool zact = zcc < MCOL && zcol < ncols;
    const int zl = zcol % A.L, zr = zcol / A.L;
    typename C::acc_t acc[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = typename C::acc_t{};
    R av[APT];
    zd x0, x1, x2;
    const int qend = A.seg_begin[sg + 1];
    RowJob cur;
    job_face(A, A.seg_begin[sg], cur);
    ROW_FETCH(cur);
    ROW_STORE(cur, 0);
    __syncthreads();
    int buf = 0;
    for (;;) {
        RowJob nxt = cur;
        bool more = true;
        nxt.k0 += KC;
        if (nxt.k0 >= nxt.kreal) {
            if (cur.q + 1 < qend) job_face(A, cur.q + 1, nxt);
            else more = false;
        }
        if (more) ROW_FETCH(nxt);
        mfma_tile<R, 2>(As[buf], Bs[buf], rt0, ct0, nrt, lane, acc);
        if (!more) break;
        ROW_STORE(nxt, buf ^ 1);
        __syncthreads();
        buf ^= 1;
        cur = nxt;
    }
    zd* pb = A.pbuf + (size_t)sg * MTM * ncols;
    const int li = lane & 15;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int rt = rt0 + 4 * u;
        if (rt >= nrt) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rc = 16 * (ct0 + v) + li, col = c0 + (rc >> 1);
            if (col >= ncols) continue;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const int row = 16 * rt + C::orow(lane, w);
                if (row < nrows) ((double*)(pb + (size_t)row * ncols + col))[rc & 1] = (double)acc[u][v][w];
            }
        }
    }
}

#undef ROW_FETCH
#undef ROW_STORE

// y rows of row chunk g = sum of its segments' partial rows, in segment order
__global__ __launch_bounds__(256) void k_reduce_mrows(MApplyArgs A, int ncols)
{
    const int g = blockIdx.x;
    const int rsz = A.row_size[g], rs0 = A.row_start[g];
    const int q = blockIdx.y * 256 + threadIdx.x;  // (row, col) with col fastest
    if (q >= 3 * rsz * ncols) return;
    const int row = q / ncols, col = q - row * ncols;
    zd s = {0.0, 0.0};
    for (int sg = A.group_seg[g]; sg < A.group_seg[g + 1]; ++sg) s += A.pbuf[((size_t)sg * MTM + row) * ncols + col];
    const size_t M = 3 * (size_t)A.K;
    const int l = col % A.L, r = col / A.L;
    A.y[((size_t)r * A.L + l) * M + 3 * (size_t)rs0 + row] = s;
}

}  // namespace

void launch_apply_mfma(const MApplyArgs& A, hipStream_t st)
{
    const int ncols = A.L * A.nrhs;
    const long long ct = (ncols + MCOL - 1) / MCOL;
    auto grid = [&](int n) {
        if ((long long)n * ct >= (1LL << 31)) throw std::invalid_argument("too many product work items");
        return dim3((unsigned)(n * ct));
    };
    if (A.nfar64 > 0) hipLaunchKernelGGL(k_far_mfma<double>, grid(A.nfar64), dim3(WGM), 0, st, A, ncols, A.far64, A.nfar64);
    if (A.nfar32 > 0) hipLaunchKernelGGL(k_far_mfma<float>, grid(A.nfar32), dim3(WGM), 0, st, A, ncols, A.far32, A.nfar32);
    BEM_HIP_TRY(hipGetLastError());
    if (A.nseg64 > 0) hipLaunchKernelGGL(k_rows_mfma<double>, grid(A.nseg64), dim3(WGM), 0, st, A, ncols, A.seg64, A.nseg64);
    if (A.nseg32 > 0) hipLaunchKernelGGL(k_rows_mfma<float>, grid(A.nseg32), dim3(WGM), 0, st, A, ncols, A.seg32, A.nseg32);
    BEM_HIP_TRY(hipGetLastError());
    if (A.ngroups > 0)
        hipLaunchKernelGGL(k_reduce_mrows, dim3(A.ngroups, (3 * MFMA_ROW_CHUNK * ncols + 255) / 256), dim3(256), 0, st, A,
                           ncols);
    BEM_HIP_TRY(hipGetLastError());
}

}  // namespace bem
