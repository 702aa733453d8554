// aca3d.hpp -- device-side data of the compressed operator and the compression launch.
#pragma once

#include "lib.hpp"

namespace bem {

constexpr int MAX_L = 256;  // largest number of frequencies of one compression

struct BlockIn {
    int rb, rs, cb, cs;  // rows [rb, rb + rs), columns [cb, cb + cs) in cluster order
    int far;             // admissible (far field): mixed precision applies
    int lowrank;         // faces by per-slice ACA + recompression (else dense faces)
};

// One face-fibre pair of a block.  kk == 0: dense face (3m x 3n row-major at face_off,
// complex128, or complex64 when fp32); kk > 0: factors Ubar (3m x kk) then Vbar (3n x kk), column-major, complex64
// (MIXED) or complex128; kk < 0: empty face.  fib_off: fibre f[L][3][3] complex128.
// sel = 1: dense-fallback face, its fibre selects frequency k only.
struct FaceDesc {
    long long face_off;
    long long fib_off;
    int kk;
    int k;
    int sel;
    int fp32;  // dense face stored as complex64 (far-field blocks of the mixed path)
};

struct BlockOut {
    int rank;
    int fallback;
    int status;    // 0 ok, 2 pool overflow
    int aca_cols;  // largest far-face rank
    long long entries;
};

struct CompressArgs {
    DevCtx c;               // element tables in cluster order
    int op;
    int mixed;
    int L;
    int nblocks;
    int kmax;               // column capacity of the per-slice ACA (multiple of 3)
    const BlockIn* blocks;
    const int* order;       // processing order (largest work first)
    FaceDesc* faces;        // [nblocks][L]
    BlockOut* out;          // [nblocks]
    char* pool;
    unsigned long long pool_cap;
    unsigned long long* pool_top;
    int* queue;
    int* err;
    double* scratch;
    size_t scratch_per_slot;  // doubles
    double eps3d, eps3d_far, eps_aca_far;
    long long* prof;          // per-phase cycle sums (built with BEM_PHASE_PROF only)
};

size_t aca_scratch_doubles(int mmax, int nmax, int kmax);
void launch_aca3d(const CompressArgs& A, int slots, hipStream_t st);

// ---------------------------------------------------------------- apply (apply.hip)

// One stored face of the apply plan.
struct ApplyFace {
    long long face_off, fib_off;
    int kk;        // 0 dense, > 0 factors
    int sel;       // selector fibre (frequency ksel only)
    int ksel;
    int block;     // index into the block table
    int fp32;      // dense face in complex64
    long long t_off;  // far faces: first row of this face's kk rows of V^H Z in the workspace [rows][ncols]
    long long zw_off; // weighted sum: offset (in zd) of this face's contracted vector (3 * cs entries)
};

struct ApplyArgs {
    const BlockIn* blocks;
    const ApplyFace* faces;
    int nfaces;
    const int* row_faces;      // faces grouped by leaf row cluster: CSR over row_ptr
    const int* row_ptr;
    const int* row_start;      // leaf row cluster start (cluster order) per group
    const int* row_size;
    int nrow_groups;
    const char* pool;
    int mixed;
    int K, L, nrhs;
    const zd* x;               // permuted input [nrhs][L][3K] (cluster order)
    zd* y;                     // permuted output
    zd* tbuf;                  // far products workspace
};

void launch_apply(const ApplyArgs& A, hipStream_t st);
void launch_permute(const zd* in, zd* out, const int* perm, int K, int L, int nrhs, int64_t in_l_stride, bool to_cluster,
                    hipStream_t st);
void launch_weighted(const ApplyArgs& A, const zd* W, zd* zw, zd* y, hipStream_t st);

}  // namespace bem
