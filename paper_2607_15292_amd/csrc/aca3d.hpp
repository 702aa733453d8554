// aca3d.hpp -- device-side data of the compressed operator and the launches of the
// compression pipeline and of the products.
#pragma once

#include "lib.hpp"

namespace bem {

constexpr int MAX_L = 256;  // largest number of frequencies of one compression
constexpr int TILE = 256;   // pairs (i, j) per workgroup in the tiled phases

// Pairs (i, j) of a block are numbered p = i * cs + j and ordered regular, near level 1,
// near level 2, self.  The face kernels take them in tiles of one class: ntr tiles of TILE
// regular pairs (k_face_dense), then tiles of 64 near-1, 16 near-2 and 4 self pairs
// (k_face_general, a group of 4 / 16 / 64 lanes per pair), so that a wavefront runs one rule.
struct BlockIn {
    int rb, rs, cb, cs;  // rows [rb, rb + rs), columns [cb, cb + cs) in cluster order
    int far;             // admissible (far field): the mixed path computes it in FP32
    int aca;             // faces compressed by the per-slice ACA + recompression pass
    int tile0, ntile;    // range of this block's pair tiles
    int ntr, nreg;       // tiles of regular pairs, number of regular pairs
    int n1, n2, n3;      // near level 1, near level 2 and self pairs
    int pair0;           // offset of the block's pair order in the pair list; -1: p = position
                         // (every pair regular)
    int f32;             // faces stored in complex64 (admissible block, mixed path)
};

// One face-fibre pair of a block.  kk == 0: dense face (3m x 3n row-major at face_off,
// complex128, or complex64 when fp32); kk > 0: factors Ubar (3m x kk) then Vbar (3n x kk),
// row-major, in the same precision, with H = Ubar Vbar^H; kk < 0: empty face.
// fib_off: fibre f[L][3][3] complex128.  sel = 1: dense-fallback face, its fibre selects
// frequency k only.
struct FaceDesc {
    long long face_off;
    long long fib_off;
    int kk;
    int k;
    int sel;
    int fp32;
};

// Per-block state of Algorithm 1 between the phases of one step.
struct BlockState {
    int k;          // current frequency k_d
    int rank;       // kept face-fibre pairs
    int active;     // iterating
    int fallback;   // dense storage requested
    int stop;       // this step ends the block (no fibre, no norm update)
    int piv;        // pivot pair of the current face
    int nextk;      // next frequency
    int aca_dense;  // faces of this block left dense by the per-slice ACA pass
    int term;       // no next frequency: the current step is the last one
    long long aca_cols;  // ACA columns (before recompression) over the faces stored as factors
    double norm2;   // ||C^(d)||_F^2
    double hn2, fmax2, s3max, fn2;
    long long entries;
    double recomp_flop;  // algorithmic flops of this block's face recompressions
    double aca_flop;     // algorithmic flops and HBM bytes of this block's per-slice ACA runs
    double aca_bytes;
    double fref;    // pivot scale: the largest 3x3 block norm of the slices C(k_1..k_d) so far
    zd pinv[9];
};

struct CompressArgs {
    DevCtx c;               // element tables in cluster order
    int op;
    int mixed;
    int L;
    int nblocks;
    int kmax;               // column capacity of the per-slice ACA scratch (multiple of 3)
    int d;                  // current step
    const BlockIn* blocks;
    FaceDesc* faces;        // [nblocks][L]
    BlockState* st;         // [nblocks]
    unsigned char* used;    // [nblocks][L]
    zd* Fda;                // [nblocks][L][9]: F_{d,a} = sum_k f_d[k] f_a[k]^H
    double* tp;             // tile partials [ntiles][8]
    const int* list;        // work list of this launch: block ids, tiles packed as (block << 12) | tile,
                            // or faces packed as (block << 8) | d
    int nlist;
    char* pool;
    unsigned long long pool_cap;
    unsigned long long* pool_top;
    int* err;
    double* scratch;
    const long long* slot_off;  // scratch slot of each list position (offset in doubles)
    int iloop;              // faces of the ACA blocks approximated inside the 3D-ACA loop (Sec. 3.1)
    long long* fac_off;     // [nblocks][L] in-loop faces: pool offset of their factors
    int* fac_kk;            // [nblocks][L] their rank (0: the face stays exact and dense)
    const long long* blk_slot;  // in-loop pass: scratch slot of each block (offset in doubles), -1 none
    int* pending;           // faces left at slot state -3 by a recompression launch (counter)
    int aca_rounds;         // resume launches allowed after intermediate recompressions (0: none)
    const int* pairs;       // pair orders of the blocks with pair0 >= 0
    const unsigned char* sel;  // blocks that k_init starts (nullptr: all); the others keep their state
    double eps3d, eps3d_far, eps_aca_far;
};

// Column cap of the per-slice ACA of an m x n (elements) face: 3 ceil(2 m n / (m + n)), the
// rank at which the ACA columns would take twice the memory of the dense face (rank-3 ACA
// steps overshoot the recompressed rank about twofold), at most 3 min(m, n).
__host__ __device__ inline int face_aca_cap(int m, int n)
{
    int s = (2 * m * n + (m + n) - 1) / (m + n);
    return 3 * (s < m ? (s < n ? s : n) : (m < n ? m : n));
}

// Scratch slot of one face in the per-slice ACA pass: ACA columns and the small matrices of
// the recompression.
// The compression pass keeps two column halves (U2, V2): an ACA that reaches the column
// capacity is recompressed into the other half and resumes from there.
struct AcaWork {
    zd *U, *V;        // 3m x kmax, 3n x kmax column-major: the current ACA columns
    zd *U2, *V2;      // the other halves (null in a one-half slot)
    zd *G, *RU, *RV;  // kmax x kmax
    zd *M, *VJ;       // kmax x kmax
    double* tol;      // [0]: absolute tolerance of the face in this slot
    int* usedrow;     // m
    int* order;       // kmax
    int* info;        // [0]: state of the face in this slot: ACA columns (> 0), -1 not resolved,
                      // -2 column capacity reached (recompress and resume), -3 resume pending,
                      // -4 done; [1]: columns to resume with; [2]: next pivot row; [3]: current
                      // half (0 or 1)
};

__device__ inline AcaWork aca_work(double* base, int m, int n, int kmax, int halves = 1)
{
    AcaWork w;
    zd* z = (zd*)base;
    w.U = z;
    z += (size_t)3 * m * kmax;
    w.U2 = halves > 1 ? z : nullptr;
    z += (size_t)(halves - 1) * 3 * m * kmax;
    w.V = z;
    z += (size_t)3 * n * kmax;
    w.V2 = halves > 1 ? z : nullptr;
    z += (size_t)(halves - 1) * 3 * n * kmax;
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
    w.tol = (double*)z;
    w.usedrow = (int*)(w.tol + kmax);
    w.order = w.usedrow + m;
    w.info = w.order + kmax;
    return w;
}

size_t aca_scratch_doubles(int mmax, int nmax, int kmax, int halves = 1);
// the slot of the compression pass: two column halves
constexpr int ACA_HALVES = 2;
// the current column half of a slot (info[3]) as U, V
__device__ inline void aca_select_half(AcaWork& w)
{
    if (w.U2 && w.info[3]) {
        zd* t = w.U;
        w.U = w.U2;
        w.U2 = t;
        t = w.V;
        w.V = w.V2;
        w.V2 = t;
    }
}
void launch_init(const CompressArgs& A, hipStream_t st);
// path: 1 / 2 regular tiles with complex64 / complex128 faces (k_face_dense, FP32 / FP64
// rule); 0 / 3 near tiles and 4 / 5 self tiles with complex128 / complex64 faces
// (k_face_general, FP64 rules)
void launch_face_dense(const CompressArgs& A, int path, hipStream_t st);
// order[off[q] ..] = pairs of block list[q] stably sorted by class (regular, near 1, near 2,
// self); counts[4 q + c] = pairs of class c (one workgroup per listed block)
void launch_classify(const DevCtx& c, const BlockIn* blocks, const int* list, const long long* off, int n,
                     int* order, int* counts, hipStream_t st);
void launch_pivot(const CompressArgs& A, hipStream_t st);
void launch_fibre(const CompressArgs& A, hipStream_t st);
void launch_cross_dense(const CompressArgs& A, hipStream_t st);
void launch_final(const CompressArgs& A, hipStream_t st);
// flags[b] = st[b].active for every block (device bytes, copied to the host between steps)
void launch_active_flags(const CompressArgs& A, unsigned char* flags, hipStream_t st);
void launch_advance(const CompressArgs& A, hipStream_t st);
void launch_final_prev(const CompressArgs& A, hipStream_t st);
void launch_fallback(const CompressArgs& A, int kf, hipStream_t st);
void launch_fallback_faces(const CompressArgs& A, int kf, hipStream_t st);
// per-slice ACA (k_face_aca); the recompression of its columns follows (k_face_recomp)
// resume = 0: first run over the listed faces; 1: the faces whose run is pending after an
// intermediate recompression (slot state -3)
void launch_face_aca(const CompressArgs& A, hipStream_t st, int resume = 0);
void launch_face_recomp(const CompressArgs& A, hipStream_t st);
// faces inside the 3D-ACA loop (Sec. 3.1): after k_face_aca + k_face_recomp of the step's faces
// (iloop = 1), move the factors to the pool (list: faces (block << 8) | d), reconstruct the
// faces and their pivot partials (list: tiles (block << 12) | t), and after the last step store
// the faces as factors (list: blocks)
void launch_iloop_store(const CompressArgs& A, hipStream_t st);
void launch_iloop_recon(const CompressArgs& A, hipStream_t st);
void launch_iloop_finish(const CompressArgs& A, hipStream_t st);
void launch_copy_segments(const char* src, char* dst, const long long* seg, int nseg, hipStream_t st);
void launch_aca_matrix(char* H, int m, int n, int fp32, double tol, int cap, int kmax, double* scratch, int* out,
                       hipStream_t st);
void launch_aca_matrix_recomp(char* H, int m, int n, int fp32, int kmax, double* scratch, int* out, hipStream_t st);

// ---------------------------------------------------------------- apply (apply.hip)

// One stored face of the apply plan.
struct ApplyFace {
    long long face_off, fib_off;
    int kk;        // 0 dense, > 0 factors
    int sel;       // selector fibre (frequency ksel only)
    int ksel;
    int block;     // index into the block table
    int fp32;      // dense face in complex64
    int pad;
    long long t_off;  // far faces: first row of this face's kk rows of V^H Z in the workspace [rows][ncols]
    long long zw_off; // weighted sum: offset (in zd) of this face's contracted vector (3 * cs entries)
};

struct ApplyArgs {
    const BlockIn* blocks;
    const ApplyFace* faces;
    int nfaces;
    const int* row_faces;      // faces grouped by row chunk: CSR over row_ptr
    const int* row_ptr;
    const int* row_start;      // row chunk start (cluster order) per group
    const int* row_size;
    int nrow_groups;
    const char* pool;
    int mixed;
    int K, L, nrhs;
    const zd* x;               // permuted input [nrhs][L][3K] (cluster order)
    zd* y;                     // permuted output
    zd* tbuf;                  // far products workspace
    const int* far_list;       // faces with kk > 0 (at most 96)
    int nfar;
    // segments of the row groups' face lists (one row-kernel workgroup per segment and column
    // tile): group, first entry of row_faces (seg_begin[nseg] = end), segments of a group
    int nseg;
    const int* seg_group;
    const int* seg_begin;
    const int* group_seg;
    zd* pbuf;                  // partial rows of the segments [nseg][3 APPLY_ROW_CHUNK][ncols]
};

constexpr int APPLY_ROW_CHUNK = 16;  // element rows per workgroup of the product (row chunks)
constexpr int APPLY_SEGMENTS = 2048;       // target number of row-kernel workgroups per column tile
constexpr int APPLY_SEGMENTS_FINE = 8192;  // the same for products of at most APPLY_FINE_COLS columns
constexpr int APPLY_FINE_COLS = 128;

// y = A(s_l)^T x with a plan grouped by column chunks (row_start / row_size: column chunks)
void launch_apply_t(const ApplyArgs& A, hipStream_t st);

// ---------------------------------------------------------------- MFMA product (mfma.hip)
// Row chunks of the product on the matrix cores: leaf clusters cut into nearly equal pieces of
// at most MFMA_ROW_CHUNK elements (126 rows: 8 MFMA row tiles); each chunk lists its
// complex128 faces, then its complex64 faces, and its segments hold faces of one precision.
// Column tiles of MFMA_COLS (rhs, l) columns.
constexpr int MFMA_ROW_CHUNK = 42;
constexpr int MFMA_COLS = 64;
constexpr int MFMA_SEGMENTS = 2048;  // target segment count for products of at most 2 column tiles

struct MApplyArgs {
    const BlockIn* blocks;
    const ApplyFace* faces;
    const char* pool;
    int K, L, nrhs;
    const zd* x;               // permuted input [nrhs][L][3K] (cluster order)
    zd* y;                     // permuted output
    zd* tbuf;                  // T = Vbar^H Z of the far faces [far_rows][ncols]
    zd* pbuf;                  // partial rows of the segments [nseg][3 MFMA_ROW_CHUNK][ncols]
    const int* row_faces;      // faces of the chunks (per chunk: complex128, then complex64)
    const int* row_start;      // chunk start (cluster order) and size (elements)
    const int* row_size;
    int ngroups;
    const int* seg_group;      // per segment: chunk, first entry of row_faces (seg_begin[nseg] = end)
    const int* seg_begin;
    const int* group_seg;      // per chunk: first segment (group_seg[ngroups] = nseg)
    int nseg;
    const int* seg64;          // segments of complex128 faces
    int nseg64;
    const int* seg32;          // segments of complex64 faces
    int nseg32;
    const int* far64;          // factored faces in complex128
    int nfar64;
    const int* far32;          // factored faces in complex64
    int nfar32;
};
void launch_apply_mfma(const MApplyArgs& A, hipStream_t st);

// Operators of a batched product: mesh-order vectors x (input) and y (output) of operator o,
// [nrhs][L][3 K], and its cluster permutation; the workspace holds all operators side by
// side, [nrhs][L][3 Ktot] with operator o at element offset koff.
constexpr int MAX_BATCH_OPS = 16;
struct BatchPerm {
    const zd* x;
    zd* y;
    const int* perm;
    int K;
    int koff;
};
struct BatchPermTable {
    BatchPerm op[MAX_BATCH_OPS];
    int nops, L, nrhs, Ktot;
};
// kmax = largest K of the table
void launch_permute_batch(const BatchPermTable& T, int kmax, zd* work, bool to_cluster, hipStream_t st);
void launch_permute(const zd* in, zd* out, const int* perm, int K, int L, int nrhs, int64_t in_l_stride, bool to_cluster,
                    hipStream_t st);
// uniform: W is one vector x [3K] standing for W_l = scale x at every l
void launch_weighted(const ApplyArgs& A, const zd* W, zd* zw, zd* y, hipStream_t st, bool uniform = false,
                     double scale = 1.0);

}  // namespace bem
