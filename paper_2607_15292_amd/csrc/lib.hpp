// lib.hpp -- internal interfaces between the libbem translation units.
#pragma once

#include "kernel.hpp"

namespace bem {

enum { OP_V = 0, OP_K = 1, OP_HK = 2, OP_TABLE = 3, OP_KL0 = 4 };  // OP_KL0 + v: linear basis, vertex v

// Everything an entry evaluation needs, passed by value to kernels.
struct DevCtx {
    Geo geo;              // element tables (mesh order, or cluster order for an operator)
    Mat<double> md;
    Mat<float> mf;
    QuadTab qt;
    Freq fr;
    const zd* table;      // OP_TABLE source, [L][K][K][9] in mesh order
    const int* perm;      // cluster position -> mesh element (table lookups); null = identity
};

// ENTRY(op, i, j, l): 3x3 block, collocation at element i, trial element j, frequency l.
// MIXED: regular pairs in FP32, special pairs in FP64.
template <bool MIXED>
__device__ __forceinline__ blk entry_dispatch(const DevCtx& c, int op, int i, int j, int l)
{
    blk out;
    if (op == OP_TABLE) {
        int K = c.geo.K;
        int mi = c.perm ? c.perm[i] : i, mj = c.perm ? c.perm[j] : j;
        const zd* src = c.table + ((size_t)((size_t)l * K + mi) * K + mj) * 9;
#pragma unroll
        for (int t = 0; t < 9; ++t) out.a[t] = src[t];
        return out;
    }
    int kop = (op == OP_V) ? 0 : 1;
    int cls = pair_class(c.geo, i, j, c.qt);
    if (cls == CLS_SELF) {
        entry_self(c.geo, kop, j, c.fr.s[l], c.fr.sinv[l], c.md, c.qt, out);
    } else if (cls != CLS_REGULAR) {
        entry_near(c.geo, kop, i, j, cls, c.fr.s[l], c.fr.sinv[l], c.md, c.qt, out);
    } else if (MIXED) {
        entry_regular<float>(c.geo, kop, i, j, c.fr.sf[l], c.fr.sinvf[l], c.mf, out);
    } else {
        entry_regular<double>(c.geo, kop, i, j, c.fr.s[l], c.fr.sinv[l], c.md, out);
    }
    if (op == OP_HK && i == j) {
        out.a[0].re += 0.5;
        out.a[4].re += 0.5;
        out.a[8].re += 0.5;
    }
    return out;
}

// ---------------------------------------------------------------- launchers (entries.hip)
void launch_entries(const DevCtx& c, int op, int mixed, int64_t n, const int32_t* i, const int32_t* j,
                    const int32_t* l, zd* out, hipStream_t st);
void launch_dense_assemble(const DevCtx& c, int op, int mixed, zd* out, hipStream_t st);
void launch_dense_apply(const zd* A, int M, int L, int nrhs, const zd* x, int64_t x_l_stride, zd* y,
                        hipStream_t st);
void launch_dense_weighted(const zd* A, int M, int L, const zd* W, zd* y, hipStream_t st);
// y = A(s_l)^T x for the stored dense slices, x, y [nrhs][L][M]
void launch_dense_apply_t(const zd* A, int M, int L, int nrhs, const zd* x, zd* y, hipStream_t st);

// ---------------------------------------------------------------- matrix-free (adjoint.hip)
// y = A(s_l) x (transpose: A(s_l)^T x) for every l with entries recomputed; mesh order
// [nrhs][L][3K]
void launch_mf_apply(const DevCtx& c, int op, bool transpose, int nrhs, const zd* x, zd* y, hipStream_t st);
// y[r][l] = (C + K_lin(s_l)) g[r][l] (free_term) or K_lin(s_l) g[r][l]: the double layer against
// the nodal hat functions, entries recomputed; g [nrhs][L][3 N] by node, y [nrhs][L][3K] by
// element (mesh order); tri [K][3] node indices
void launch_mf_apply_kl(const DevCtx& c, const int* tri, int nnodes, int nrhs, const zd* g, zd* y, bool free_term,
                        hipStream_t st);
size_t adjoint_work_doubles(int K);
void launch_adjoint_v(const DevCtx& c, int nrhs, const zd* w, const zd* x, double* work, double** sums, double** tiles,
                      int* ntiles, double** self_out, hipStream_t st);
void launch_adjoint_k(const DevCtx& c, bool free_term, int nrhs, const zd* w, const zd* x, double* work, double** sums,
                      double** tiles, int* ntiles, double** self_out, hipStream_t st);

}  // namespace bem
