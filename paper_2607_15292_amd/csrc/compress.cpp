// compress.cpp -- host driver of the compression (partition, cluster-ordered tables,
// persistent 3D-ACA launch, statistics) and of the compressed products (apply plan).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <cstdio>

#include "aca3d.hpp"
#include "host.hpp"

namespace bem {

// Plan of the product on the matrix cores (mfma.hip): row chunks of at most MFMA_ROW_CHUNK
// elements, each with its complex128 faces, then its complex64 faces.
struct MPlan {
    std::vector<int> flat, ptr, nf64, start, size, far64, far32;
    DevBuf flat_dev, start_dev, size_dev, far_dev;
    struct Segs {
        DevBuf dev;  // [nseg] chunk, [nseg + 1] first face, [ngroups + 1] first segment, [n64], [n32]
        int nseg = 0, n64 = 0, n32 = 0;
    };
    Segs fine, coarse;  // fine: products of at most 2 column tiles
    int ngroups = 0;
};

struct CompressedOp {
    Partition part;
    DevGeo geo;                 // element tables in cluster order
    DevBuf perm_dev;            // [K] cluster position -> mesh element
    DevBuf blocks_dev;          // BlockIn[nb]
    DevBuf faces_dev;           // FaceDesc[nb][L]
    DevBuf pool;                // faces, factors, fibres (offsets of FaceDesc are from its base)
    std::vector<std::unique_ptr<DevBuf>> extra_pools;  // pools of further block groups, above it
    std::vector<BlockIn> blocks;
    std::vector<FaceDesc> faces;
    std::vector<BlockState> st;
    // apply plan
    std::vector<ApplyFace> af;
    std::vector<int> h_flat, h_ptr, h_start, h_size, h_far;  // row groups and far faces (host copy)
    DevBuf af_dev, rowfaces_dev, rowptr_dev, rowstart_dev, rowsize_dev, farlist_dev;
    DevBuf seg_dev;             // segments: [nseg] group, [nseg + 1] face ranges, [ngroups + 1] group ranges
    DevBuf segf_dev;            // finer segments for products of few columns (nsegf of them)
    int nsegf = 0;
    int ngroups = 0;
    int nseg = 0;
    int nfar = 0;               // factored faces
    long long far_rows = 0;     // sum of kk over far faces
    long long zw_total = 0;     // sum of 3 cs over faces
    MPlan mp;                   // plan of the product (matrix cores)
    DevBuf work;                // apply workspace (grown on demand)
    // plan of the transposed product (column chunks), built on first use
    bool t_built = false;
    int nseg_t = 0;
    DevBuf rowfaces_t_dev, rowptr_t_dev, seg_t_dev;
    int mixed = 0, L = 0, K = 0;
    int ngroups_c = 1;          // block groups of the compression
};

void destroy_compressed(CompressedOp* c) { delete c; }

namespace {

using Err = ApiError;
constexpr int KMAX_ACA = 96;       // column capacity of the per-slice ACA scratch
// Algorithmic flop counts of the face kernels: one kernel evaluation at one quadrature
// point (distance, A and B or A', B', the tensor terms; complex mul = 6, add = 2, exp /
// sin / cos counted as one flop each), and one residual update H_a[i,j] f_a[k] (27 complex
// multiply-adds = 216 flops).
constexpr double QPTS_REGULAR = 7.0;
constexpr double FLOPS_RESIDUAL = 216.0;
double flops_eval(int op) { return op == BEM_OP_V ? 125.0 : (op == BEM_OP_TABLE ? 0.0 : 236.0); }
constexpr size_t ACA_SLOTS = 8192;  // faces per launch of the per-slice ACA pass (scratch slots)
constexpr size_t ACA_SCRATCH_BYTES = (size_t)16 << 30;  // scratch of one such launch, at most
constexpr int POOL_STEPS0 = 32;     // 3D-ACA steps of every block in the initial pool

// Segments: each row group's face list cut into pieces of about equal work (the staged inner
// dimension: 3 cs for a dense face, kk for factors, plus a per-face overhead), about target
// pieces in all; partial sums are added in segment order.  segbuf = [nseg] group, [nseg + 1]
// first face entry, [ngroups + 1] first segment of each group.
std::vector<int> make_segments(const std::vector<ApplyFace>& af, const std::vector<BlockIn>& blocks,
                               const std::vector<int>& ptr, const std::vector<int>& flat, int target, int* nseg_out,
                               bool transpose = false)
{
    const int ngroups = (int)ptr.size() - 1;
    auto cost = [&](int fi) {
        const ApplyFace& a = af[fi];
        const BlockIn& B = blocks[a.block];
        return (double)(a.kk > 0 ? a.kk : 3 * (transpose ? B.rs : B.cs)) + 24.0;
    };
    double total = 0.0;
    for (int fi : flat) total += cost(fi);
    const double per = std::max(1.0, total / std::max(target, 1));
    std::vector<int> sgroup, sbeg, gseg(ngroups + 1, 0);
    for (int g = 0; g < ngroups; ++g) {
        double cg = 0.0;
        for (int q = ptr[g]; q < ptr[g + 1]; ++q) cg += cost(flat[q]);
        const int ns = std::max(1, (int)std::lround(cg / per));
        const double tgt = cg / ns;
        int q = ptr[g];
        for (int k = 0; k < ns; ++k) {
            sgroup.push_back(g);
            sbeg.push_back(q);
            double acc = 0.0;
            while (q < ptr[g + 1] && (k == ns - 1 || acc == 0.0 || acc + 0.5 * cost(flat[q]) < tgt)) acc += cost(flat[q++]);
        }
        gseg[g + 1] = (int)sgroup.size();
    }
    *nseg_out = (int)sgroup.size();
    std::vector<int> segbuf;
    segbuf.insert(segbuf.end(), sgroup.begin(), sgroup.end());
    segbuf.insert(segbuf.end(), sbeg.begin(), sbeg.end());
    segbuf.push_back(ptr[ngroups]);
    segbuf.insert(segbuf.end(), gseg.begin(), gseg.end());
    return segbuf;
}

void build_apply_plan(CompressedOp& C, hipStream_t st)
{
    const int L = C.L;
    const int nb = (int)C.blocks.size();
    C.af.clear();
    std::vector<std::vector<int>> faces_of_block(nb);
    long long trow = 0, zw = 0;
    for (int b = 0; b < nb; ++b) {
        for (int d = 0; d < C.st[b].rank; ++d) {
            const FaceDesc& f = C.faces[(size_t)b * L + d];
            if (f.kk < 0) continue;
            ApplyFace a;
            a.face_off = f.face_off;
            a.fib_off = f.fib_off;
            a.kk = f.kk;
            a.sel = f.sel;
            a.ksel = f.k;
            a.block = b;
            a.fp32 = f.fp32;
            a.pad = 0;
            a.t_off = 0;
            if (f.kk > 0) {
                a.t_off = trow;
                trow += f.kk;
            }
            a.zw_off = zw;
            zw += 3LL * C.blocks[b].cs;
            faces_of_block[b].push_back((int)C.af.size());
            C.af.push_back(a);
        }
    }
    C.far_rows = trow;
    C.zw_total = zw;
    // row chunks: leaves of the cluster tree cut into pieces of at most APPLY_ROW_CHUNK
    std::vector<int> cstart, csize;
    for (const Cluster& n : C.part.nodes)
        if (n.child[0] < 0)
            for (int s = 0; s < n.size; s += APPLY_ROW_CHUNK) {
                cstart.push_back(n.begin + s);
                csize.push_back(std::min(APPLY_ROW_CHUNK, n.size - s));
            }
    std::vector<int> far;
    for (size_t f = 0; f < C.af.size(); ++f)
        if (C.af[f].kk > 0) {
            if (C.af[f].kk > 96) throw ApiError(BEM_ERR_ARG, "factored face rank above 96");
            far.push_back((int)f);
        }
    C.nfar = (int)far.size();
    std::vector<int> order(cstart.size());
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int a, int b) { return cstart[a] < cstart[b]; });
    std::vector<int> s2(order.size()), z2(order.size());
    for (size_t i = 0; i < order.size(); ++i) {
        s2[i] = cstart[order[i]];
        z2[i] = csize[order[i]];
    }
    C.ngroups = (int)s2.size();
    std::vector<std::vector<int>> lists(C.ngroups);
    for (int b = 0; b < nb; ++b) {
        const BlockIn& B = C.blocks[b];
        auto it = std::lower_bound(s2.begin(), s2.end(), B.rb);
        for (; it != s2.end() && *it < B.rb + B.rs; ++it) {
            int g = (int)(it - s2.begin());
            for (int fi : faces_of_block[b]) lists[g].push_back(fi);
        }
    }
    std::vector<int> ptr(C.ngroups + 1, 0), flat;
    for (int g = 0; g < C.ngroups; ++g) {
        ptr[g + 1] = ptr[g] + (int)lists[g].size();
        flat.insert(flat.end(), lists[g].begin(), lists[g].end());
    }
    std::vector<int> segbuf = make_segments(C.af, C.blocks, ptr, flat, APPLY_SEGMENTS, &C.nseg);
    auto up = [&](DevBuf& d, const void* src, size_t bytes) {
        d.alloc(std::max<size_t>(bytes, 16));
        if (bytes) BEM_HIP_TRY(hipMemcpyAsync(d.p, src, bytes, hipMemcpyHostToDevice, st));
    };
    up(C.af_dev, C.af.data(), C.af.size() * sizeof(ApplyFace));
    up(C.rowfaces_dev, flat.data(), flat.size() * sizeof(int));
    up(C.rowptr_dev, ptr.data(), ptr.size() * sizeof(int));
    up(C.rowstart_dev, s2.data(), s2.size() * sizeof(int));
    up(C.rowsize_dev, z2.data(), z2.size() * sizeof(int));
    up(C.farlist_dev, far.data(), far.size() * sizeof(int));
    up(C.seg_dev, segbuf.data(), segbuf.size() * sizeof(int));
    std::vector<int> segf = make_segments(C.af, C.blocks, ptr, flat, APPLY_SEGMENTS_FINE, &C.nsegf);
    up(C.segf_dev, segf.data(), segf.size() * sizeof(int));
    BEM_HIP_TRY(hipStreamSynchronize(st));
    C.h_flat = std::move(flat);
    C.h_ptr = std::move(ptr);
    C.h_start = std::move(s2);
    C.h_size = std::move(z2);
    C.h_far = std::move(far);
}

// Segments of the product on the matrix cores: the complex128 faces and the complex64 faces
// of every chunk cut into pieces of about equal work (staged k per face: 3 cs for a dense face,
// kk for factors, plus a per-face overhead; complex128 work counts twice, the FP64 MFMA rate
// being half the FP32 one), about target pieces in all.  Partial sums are added in segment
// order.  Returns [nseg] chunk, [nseg + 1] first face entry, [ngroups + 1] first segment of
// each chunk, [n64] complex128 segments, [n32] complex64 segments.
std::vector<int> make_msegments(const std::vector<ApplyFace>& af, const std::vector<BlockIn>& blocks,
                                const std::vector<int>& ptr, const std::vector<int>& nf64, const std::vector<int>& flat,
                                int target, int* nseg, int* n64, int* n32)
{
    const int ngroups = (int)ptr.size() - 1;
    auto cost = [&](int fi) {
        const ApplyFace& a = af[fi];
        return (a.kk > 0 ? (double)a.kk : 3.0 * blocks[a.block].cs) + 16.0;
    };
    double total = 0.0;
    for (int g = 0; g < ngroups; ++g)
        for (int q = ptr[g]; q < ptr[g + 1]; ++q) total += cost(flat[q]) * (q < ptr[g] + nf64[g] ? 2.0 : 1.0);
    const double per = std::max(1.0, total / std::max(target, 1));
    std::vector<int> sgroup, sbeg, s64, s32, gseg(ngroups + 1, 0);
    for (int g = 0; g < ngroups; ++g) {
        for (int p = 0; p < 2; ++p) {
            const int b = ptr[g] + (p ? nf64[g] : 0), e = p ? ptr[g + 1] : ptr[g] + nf64[g];
            if (b >= e) continue;
            const double w = p ? 1.0 : 2.0;
            double cg = 0.0;
            for (int q = b; q < e; ++q) cg += w * cost(flat[q]);
            const int ns = std::max(1, (int)std::lround(cg / per));
            const double tgt = cg / ns;
            int q = b;
            for (int k = 0; k < ns && q < e; ++k) {
                (p ? s32 : s64).push_back((int)sgroup.size());
                sgroup.push_back(g);
                sbeg.push_back(q);
                double acc = 0.0;
                while (q < e && (k == ns - 1 || acc == 0.0 || acc + 0.5 * w * cost(flat[q]) < tgt)) acc += w * cost(flat[q++]);
            }
        }
        gseg[g + 1] = (int)sgroup.size();
    }
    *nseg = (int)sgroup.size();
    *n64 = (int)s64.size();
    *n32 = (int)s32.size();
    std::vector<int> segbuf;
    segbuf.insert(segbuf.end(), sgroup.begin(), sgroup.end());
    segbuf.insert(segbuf.end(), sbeg.begin(), sbeg.end());
    segbuf.push_back(ptr[ngroups]);
    segbuf.insert(segbuf.end(), gseg.begin(), gseg.end());
    segbuf.insert(segbuf.end(), s64.begin(), s64.end());
    segbuf.insert(segbuf.end(), s32.begin(), s32.end());
    return segbuf;
}

void upload_ints(DevBuf& d, const std::vector<int>& v, hipStream_t st)
{
    d.alloc(std::max<size_t>(v.size() * sizeof(int), 16));
    if (!v.empty()) BEM_HIP_TRY(hipMemcpyAsync(d.p, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, st));
}

void set_msegments(MPlan::Segs& S, const std::vector<ApplyFace>& af, const std::vector<BlockIn>& blocks,
                   const MPlan& P, int target, hipStream_t st)
{
    upload_ints(S.dev, make_msegments(af, blocks, P.ptr, P.nf64, P.flat, target, &S.nseg, &S.n64, &S.n32), st);
}

// Chunks: leaves of the cluster tree cut into nearly equal pieces of at most MFMA_ROW_CHUNK
// elements, in cluster order; each gets the faces of the blocks whose rows cover it,
// complex128 first.
void build_mplan(CompressedOp& C, hipStream_t st)
{
    MPlan& P = C.mp;
    std::vector<std::pair<int, int>> ch;
    for (const Cluster& n : C.part.nodes)
        if (n.child[0] < 0) {
            const int pieces = (n.size + MFMA_ROW_CHUNK - 1) / MFMA_ROW_CHUNK;
            for (int q = 0, s0 = 0; q < pieces; ++q) {
                const int sz = (n.size - s0) / (pieces - q);
                ch.push_back({n.begin + s0, sz});
                s0 += sz;
            }
        }
    std::sort(ch.begin(), ch.end());
    P.ngroups = (int)ch.size();
    P.start.resize(P.ngroups);
    P.size.resize(P.ngroups);
    for (int g = 0; g < P.ngroups; ++g) {
        P.start[g] = ch[g].first;
        P.size[g] = ch[g].second;
    }
    const int nb = (int)C.blocks.size();
    std::vector<std::vector<int>> of_block(nb);
    for (size_t f = 0; f < C.af.size(); ++f) of_block[C.af[f].block].push_back((int)f);
    std::vector<std::vector<int>> l64(P.ngroups), l32(P.ngroups);
    for (int b = 0; b < nb; ++b) {
        const BlockIn& B = C.blocks[b];
        auto it = std::lower_bound(P.start.begin(), P.start.end(), B.rb);
        for (; it != P.start.end() && *it < B.rb + B.rs; ++it) {
            const int g = (int)(it - P.start.begin());
            for (int fi : of_block[b]) (C.af[fi].fp32 ? l32 : l64)[g].push_back(fi);
        }
    }
    P.flat.clear();
    P.ptr.assign(1, 0);
    P.nf64.assign(P.ngroups, 0);
    for (int g = 0; g < P.ngroups; ++g) {
        P.nf64[g] = (int)l64[g].size();
        P.flat.insert(P.flat.end(), l64[g].begin(), l64[g].end());
        P.flat.insert(P.flat.end(), l32[g].begin(), l32[g].end());
        P.ptr.push_back((int)P.flat.size());
    }
    P.far64.clear();
    P.far32.clear();
    for (size_t f = 0; f < C.af.size(); ++f)
        if (C.af[f].kk > 0) (C.af[f].fp32 ? P.far32 : P.far64).push_back((int)f);
    std::vector<int> far = P.far64;
    far.insert(far.end(), P.far32.begin(), P.far32.end());
    upload_ints(P.flat_dev, P.flat, st);
    upload_ints(P.start_dev, P.start, st);
    upload_ints(P.size_dev, P.size, st);
    upload_ints(P.far_dev, far, st);
    set_msegments(P.fine, C.af, C.blocks, P, MFMA_SEGMENTS, st);
    set_msegments(P.coarse, C.af, C.blocks, P, std::max(P.ngroups, 256), st);
    BEM_HIP_TRY(hipStreamSynchronize(st));
}

// Arguments of the product on the matrix cores for segments S; the workspace pointers are
// set by the caller.
MApplyArgs margs(const MPlan& P, const MPlan::Segs& S, const DevBuf& blocks_dev, const DevBuf& af_dev,
                 const char* pool, int K, int L, int nrhs)
{
    MApplyArgs A{};
    A.blocks = blocks_dev.as<BlockIn>();
    A.faces = af_dev.as<ApplyFace>();
    A.pool = pool;
    A.K = K;
    A.L = L;
    A.nrhs = nrhs;
    A.row_faces = P.flat_dev.as<int>();
    A.row_start = P.start_dev.as<int>();
    A.row_size = P.size_dev.as<int>();
    A.ngroups = P.ngroups;
    A.nseg = S.nseg;
    A.seg_group = S.dev.as<int>();
    A.seg_begin = A.seg_group + S.nseg;
    A.group_seg = A.seg_begin + S.nseg + 1;
    A.seg64 = A.group_seg + P.ngroups + 1;
    A.nseg64 = S.n64;
    A.seg32 = A.seg64 + S.n64;
    A.nseg32 = S.n32;
    A.far64 = P.far_dev.as<int>();
    A.nfar64 = (int)P.far64.size();
    A.far32 = A.far64 + P.far64.size();
    A.nfar32 = (int)P.far32.size();
    return A;
}

ApplyArgs plan_args(const CompressedOp& C, int nrhs)
{
    ApplyArgs A{};
    A.blocks = C.blocks_dev.as<BlockIn>();
    A.faces = C.af_dev.as<ApplyFace>();
    A.nfaces = (int)C.af.size();
    A.row_faces = C.rowfaces_dev.as<int>();
    A.row_ptr = C.rowptr_dev.as<int>();
    A.row_start = C.rowstart_dev.as<int>();
    A.row_size = C.rowsize_dev.as<int>();
    A.nrow_groups = C.ngroups;
    A.pool = C.pool.as<char>();
    A.mixed = C.mixed;
    A.K = C.K;
    A.L = C.L;
    A.nrhs = nrhs;
    A.far_list = C.farlist_dev.as<int>();
    A.nfar = C.nfar;
    // few columns: the finer segments keep enough row workgroups in flight
    const bool fine = (size_t)C.L * nrhs <= (size_t)APPLY_FINE_COLS;
    A.nseg = fine ? C.nsegf : C.nseg;
    A.seg_group = (fine ? C.segf_dev : C.seg_dev).as<int>();
    A.seg_begin = A.seg_group + A.nseg;
    A.group_seg = A.seg_begin + A.nseg + 1;
    return A;
}

// True when no pair (i, j) of the admissible block d can take the self or a near rule:
// the boxes of the collocation points (rows) and of the element centroids (columns) are
// farther apart than near_r2 times the longest edge of any column element.  Same
// comparison as the pair classification, conservatively on the boxes.
bool all_pairs_regular(const HostGeo& g, const std::vector<int>& perm, const bem_quad& q, const BlockDesc& d)
{
    if (d.rb < d.cb + d.cs && d.cb < d.rb + d.rs) return false;  // shared elements: self pairs
    if (!q.near_on) return true;
    double lo[2][3], hi[2][3], l2 = 0.0;
    for (int s = 0; s < 2; ++s) {
        const int b0 = s ? d.cb : d.rb, n = s ? d.cs : d.rs;
        for (int c = 0; c < 3; ++c) {
            lo[s][c] = 1e300;
            hi[s][c] = -1e300;
        }
        for (int t = 0; t < n; ++t) {
            const int e = perm[b0 + t];
            const double x[3] = {g.cx[e], g.cy[e], g.cz[e]};
            for (int c = 0; c < 3; ++c) {
                lo[s][c] = std::min(lo[s][c], x[c]);
                hi[s][c] = std::max(hi[s][c], x[c]);
            }
            if (s) l2 = std::max(l2, g.lmax2[e]);
        }
    }
    double d2 = 0.0;
    for (int c = 0; c < 3; ++c) {
        const double gap = std::max({0.0, lo[0][c] - hi[1][c], lo[1][c] - hi[0][c]});
        d2 += gap * gap;
    }
    const double r2 = std::max(q.near_r1, q.near_r2);
    return d2 > 1.0001 * r2 * r2 * l2;
}

// Upload a host list into the device list buffer at element offset `at`; returns pointer.
const int* put_list(DevBuf& buf, size_t at, const std::vector<int>& v, hipStream_t st)
{
    int* p = buf.as<int>() + at;
    if (!v.empty()) BEM_HIP_TRY(hipMemcpyAsync(p, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, st));
    return p;
}

}  // namespace

int compress_impl(bem_ctx* ctx, int op, const bem_aca_opts& o, bem_op* out)
{
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = ctx->stream;
    const int K = ctx->hgeo.K, L = ctx->freq.L;
    if (L > MAX_L) throw Err(BEM_ERR_ARG, "compression supports at most 256 frequencies");
    CompressedOp* C = new CompressedOp();
    out->comp = C;
    C->mixed = o.prec == BEM_PREC_MIXED;
    C->L = L;
    C->K = K;
    build_partition(ctx->hgeo, o.eta, o.leaf, C->part);
    C->geo.upload(ctx->hgeo, C->part.perm.data(), st);
    C->perm_dev.alloc(sizeof(int) * K);
    BEM_HIP_TRY(hipMemcpyAsync(C->perm_dev.p, C->part.perm.data(), sizeof(int) * K, hipMemcpyHostToDevice, st));
    const int nb = (int)C->part.blocks.size();
    if (nb >= (1 << 19)) throw Err(BEM_ERR_ARG, "too many blocks for the compression work lists");
    C->blocks.resize(nb);
    int mmax = 1, nmax = 1, kmax = 6;
    int64_t n_far = 0, n_aca = 0;
    int ntiles = 0;
    std::vector<int> cls_blocks;  // blocks with near or self pairs: classified on the device
    for (int b = 0; b < nb; ++b) {
        const BlockDesc& d = C->part.blocks[b];
        const int aca = d.far && std::min(d.rs, d.cs) > o.far_dense_max;
        const int f32 = C->mixed && d.far;
        C->blocks[b] = BlockIn{d.rb, d.rs, d.cb, d.cs, d.far, aca, 0, 0, 0, d.rs * d.cs, 0, 0, 0, -1, f32};
        const bool reg = op == BEM_OP_TABLE || (d.far && all_pairs_regular(ctx->hgeo, C->part.perm, ctx->quad, d));
        if (!reg) cls_blocks.push_back(b);
        n_far += d.far;
        if (aca) {
            ++n_aca;
            mmax = std::max(mmax, d.rs);
            nmax = std::max(nmax, d.cs);
            kmax = std::max(kmax, face_aca_cap(d.rs, d.cs));
        }
    }
    // pair orders: regular pairs first, then the near and self pairs sorted by class
    DevBuf pairs_dev;
    if (!cls_blocks.empty()) {
        std::vector<long long> off(cls_blocks.size() + 1, 0);
        for (size_t q = 0; q < cls_blocks.size(); ++q) {
            const BlockIn& B = C->blocks[cls_blocks[q]];
            off[q + 1] = off[q] + (long long)B.rs * B.cs;
        }
        if (off.back() >= (1LL << 31)) throw Err(BEM_ERR_ARG, "pair list too long");
        DevBuf off_d, lst_d, cnt_d;
        off_d.alloc(sizeof(long long) * off.size());
        lst_d.alloc(sizeof(int) * cls_blocks.size());
        cnt_d.alloc(sizeof(int) * 4 * cls_blocks.size());
        pairs_dev.alloc(sizeof(int) * std::max<long long>(off.back(), 4));
        C->blocks_dev.alloc(sizeof(BlockIn) * nb);
        BEM_HIP_TRY(hipMemcpyAsync(C->blocks_dev.p, C->blocks.data(), sizeof(BlockIn) * nb, hipMemcpyHostToDevice, st));
        BEM_HIP_TRY(hipMemcpyAsync(off_d.p, off.data(), sizeof(long long) * off.size(), hipMemcpyHostToDevice, st));
        BEM_HIP_TRY(hipMemcpyAsync(lst_d.p, cls_blocks.data(), sizeof(int) * cls_blocks.size(), hipMemcpyHostToDevice, st));
        launch_classify(ctx->devctx(C->geo.geo, C->perm_dev.as<int>()), C->blocks_dev.as<BlockIn>(), lst_d.as<int>(),
                        off_d.as<long long>(), (int)cls_blocks.size(), pairs_dev.as<int>(), cnt_d.as<int>(), st);
        std::vector<int> cnt(4 * cls_blocks.size());
        BEM_HIP_TRY(hipMemcpyAsync(cnt.data(), cnt_d.p, sizeof(int) * cnt.size(), hipMemcpyDeviceToHost, st));
        BEM_HIP_TRY(hipStreamSynchronize(st));
        for (size_t q = 0; q < cls_blocks.size(); ++q) {
            BlockIn& B = C->blocks[cls_blocks[q]];
            B.pair0 = (int)off[q];
            B.nreg = cnt[4 * q];
            B.n1 = cnt[4 * q + 1];
            B.n2 = cnt[4 * q + 2];
            B.n3 = cnt[4 * q + 3];
        }
    }
    for (int b = 0; b < nb; ++b) {
        BlockIn& B = C->blocks[b];
        B.ntr = (B.nreg + TILE - 1) / TILE;
        B.ntile = B.ntr + (B.n1 + TILE / 4 - 1) / (TILE / 4) + (B.n2 + TILE / 16 - 1) / (TILE / 16) +
                  (B.n3 + TILE / 64 - 1) / (TILE / 64);
        if (B.ntile >= 4096) throw Err(BEM_ERR_ARG, "block too large for the tile lists (raise leaf or lower eta)");
        B.tile0 = ntiles;
        ntiles += B.ntile;
    }
    kmax = std::min(kmax, KMAX_ACA);
    DevBuf aux, st_dev, used_dev, fda_dev, tp_dev, list_dev;
    if (!C->blocks_dev.p) C->blocks_dev.alloc(sizeof(BlockIn) * nb);
    BEM_HIP_TRY(hipMemcpyAsync(C->blocks_dev.p, C->blocks.data(), sizeof(BlockIn) * nb, hipMemcpyHostToDevice, st));
    aux.alloc(256);
    int* err_dev = aux.as<int>();
    unsigned long long* top_dev = (unsigned long long*)(aux.as<char>() + 64);
    C->faces_dev.alloc(sizeof(FaceDesc) * (size_t)nb * L);
    st_dev.alloc(sizeof(BlockState) * nb);
    used_dev.alloc((size_t)nb * L);
    fda_dev.alloc(sizeof(zd) * 9 * (size_t)nb * L);
    tp_dev.alloc(sizeof(double) * 8 * (size_t)ntiles);
    list_dev.alloc(sizeof(int) * std::max<size_t>(3 * (size_t)ntiles + 2 * (size_t)nb + 64, (size_t)n_aca * L + 64));
    // faces inside the loop (Sec. 3.1 order): the factors of each face, a work list of faces,
    // tiles and scratch slots, and one scratch slot per ACA block of a launch chunk
    const bool iloop = o.face_order == BEM_FACES_IN_LOOP && n_aca > 0;
    DevBuf facoff_dev, fackk_dev, il_list_dev, il_slot_dev;
    if (iloop) {
        facoff_dev.alloc(sizeof(long long) * (size_t)nb * L);
        fackk_dev.alloc(sizeof(int) * (size_t)nb * L);
        BEM_HIP_TRY(hipMemsetAsync(fackk_dev.p, 0, sizeof(int) * (size_t)nb * L, st));
        il_list_dev.alloc(sizeof(int) * ((size_t)n_aca + (size_t)ntiles + 64));
        il_slot_dev.alloc(sizeof(long long) * ((size_t)n_aca + 64));
    }
    // pool of faces and fibres: sized for POOL_STEPS0 steps of every block (or by the caller)
    // and grown between steps, by a copy of its used part, when the allocations of the next
    // step might not fit
    auto step_bytes = [&](int b) -> size_t {  // one face + fibre of block b as pool_alloc rounds
        const BlockIn& B = C->blocks[b];
        const size_t zs = B.f32 ? sizeof(zf) : sizeof(zd);
        const size_t fb = (zs * 9 * (size_t)B.rs * B.cs + 15) & ~(size_t)15;
        const size_t fac = iloop && B.aca ? fb + 256 : 0;  // the factors of an in-loop face
        return (fb + sizeof(zd) * 9 * (size_t)L + 255 + fac) & ~(size_t)255;
    };
    auto avail = [&]() {
        size_t fr = 0, tot = 0;
        BEM_HIP_TRY(hipMemGetInfo(&fr, &tot));
        return fr + ctx->cache.cached;
    };
    const bool auto_pool = o.pool_bytes == 0;
    const size_t steps0 = (size_t)std::min(L, POOL_STEPS0);
    C->pool.cache = &ctx->cache;
    C->work.cache = &ctx->cache;
    BEM_HIP_TRY(hipStreamSynchronize(st));
    hipEvent_t ev0, ev1, ev2, evf0, evf1;
    BEM_HIP_TRY(hipEventCreate(&ev0));
    BEM_HIP_TRY(hipEventCreate(&ev1));
    BEM_HIP_TRY(hipEventCreate(&ev2));
    BEM_HIP_TRY(hipEventCreate(&evf0));
    BEM_HIP_TRY(hipEventCreate(&evf1));
    double face_ms = 0.0, face_flop = 0.0, face_bytes = 0.0;
    int64_t face_launches = 0, face_pairs = 0;
    float kms = 0.f, aca_ms = 0.f;
    double recomp_ms = 0.0, aca_kernel_ms = 0.0;
    int64_t recomp_launches = 0, aca_launches = 0;
    int err = 0;
    std::vector<BlockState>& S = C->st;
    S.resize(nb);
    CompressArgs A;
    // grows the pool (between steps, stream idle) so that `need` more bytes fit
    auto ensure_pool = [&](CompressArgs& Ar, size_t need) {
        unsigned long long top = 0;
        BEM_HIP_TRY(hipMemcpy(&top, top_dev, sizeof(top), hipMemcpyDeviceToHost));
        if (top + need <= Ar.pool_cap) return;
        if (!auto_pool)
            throw Err(BEM_ERR_NOMEM, "compression pool of " + std::to_string(Ar.pool_cap) +
                                         " bytes is too small; raise pool_bytes or pass 0");
        size_t want = std::max<size_t>((size_t)(1.5 * (double)Ar.pool_cap), (size_t)top + 2 * need);
        want = std::min<size_t>(want, (size_t)(0.9 * (double)avail()));  // the old pool stays alive during the copy
        if (want < top + need) throw Err(BEM_ERR_NOMEM, "device memory exhausted by the compression pool");
        DevBuf np(&ctx->cache);
        np.alloc(want);
        BEM_HIP_TRY(hipMemcpyAsync(np.p, C->pool.p, top, hipMemcpyDeviceToDevice, st));
        BEM_HIP_TRY(hipStreamSynchronize(st));
        C->pool.swap(np);
        np.release();
        Ar.pool = C->pool.as<char>();
        Ar.pool_cap = C->pool.bytes;
    };
    BEM_HIP_TRY(hipMemsetAsync(aux.p, 0, 256, st));
    BEM_HIP_TRY(hipMemsetAsync(C->faces_dev.p, 0, sizeof(FaceDesc) * (size_t)nb * L, st));
    A = CompressArgs{};
    A.c = ctx->devctx(C->geo.geo, C->perm_dev.as<int>());
    A.op = op;
    A.mixed = C->mixed;
    A.L = L;
    A.nblocks = nb;
    A.kmax = kmax;
    A.d = 0;
    A.blocks = C->blocks_dev.as<BlockIn>();
    A.faces = C->faces_dev.as<FaceDesc>();
    A.st = st_dev.as<BlockState>();
    A.used = used_dev.as<unsigned char>();
    A.Fda = fda_dev.as<zd>();
    A.tp = tp_dev.as<double>();
    A.list = nullptr;
    A.nlist = 0;
    A.pool = C->pool.as<char>();
    A.pool_cap = C->pool.bytes;
    A.pool_top = top_dev;
    A.err = err_dev;
    A.pending = (int*)(aux.as<char>() + 128);
    A.aca_rounds = o.aca_rounds;
    A.scratch = nullptr;
    A.slot_off = nullptr;
    A.iloop = 0;
    A.fac_off = iloop ? facoff_dev.as<long long>() : nullptr;
    A.fac_kk = iloop ? fackk_dev.as<int>() : nullptr;
    A.blk_slot = nullptr;
    A.pairs = pairs_dev.as<int>();
    A.eps3d = o.eps3d;
    A.eps3d_far = C->mixed ? std::max(o.eps3d, o.mixed_eps_floor) : o.eps3d;
    A.eps_aca_far = C->mixed ? std::max(o.eps_aca, o.mixed_eps_floor) : o.eps_aca;
    BEM_HIP_TRY(hipEventRecord(ev0, st));
    // Block groups: when the faces of every block (POOL_STEPS0 steps each) would not fit the
    // memory, the blocks are compressed group after group.  Each group runs phases A to C in
    // the working pool (reused by the next group) and keeps its compacted pool; blocks of
    // other groups are inactive meanwhile (their states start at zero and k_init skips them).
    std::vector<std::unique_ptr<DevBuf>> gpools;
    std::vector<std::vector<int>> gblk;
    std::vector<unsigned char> selh((size_t)nb, 0);
    DevBuf sel_dev;
    sel_dev.alloc((size_t)nb + 64);
    BEM_HIP_TRY(hipMemsetAsync(st_dev.p, 0, sizeof(BlockState) * nb, st));
    C->faces.resize((size_t)nb * L);
    std::vector<FaceDesc> fh((size_t)nb * L);
    std::vector<int> tiles, act;
    face_ms = 0.0;
    face_launches = 0;
    face_pairs = 0;
    face_flop = 0.0;
    face_bytes = 0.0;
    // auto pool: one group if the faces of all blocks fit 60 % of the free memory; otherwise
    // groups in a working pool of 30 %, the rest left to the compacted pools of the groups
    size_t est_all = 0;
    for (int b = 0; b < nb; ++b) est_all += step_bytes(b) * steps0;
    const double pool_frac = est_all <= (size_t)(0.6 * (double)avail()) ? 0.6 : 0.3;
    for (int gpos = 0; gpos < nb;) {
    std::vector<int> grp;
    size_t pool_bytes = 0;
    {
        // the working pool of the previous group is reused: it counts as available
        const size_t budget = auto_pool ? std::max((size_t)C->pool.bytes, (size_t)(pool_frac * (double)avail()))
                                        : (size_t)o.pool_bytes;
        size_t est = 0, gstep = 0;
        while (gpos < nb) {
            const size_t e = step_bytes(gpos) * steps0;
            if (!grp.empty() && est + e > budget) break;
            est += e;
            gstep += step_bytes(gpos);
            grp.push_back(gpos++);
        }
        pool_bytes = auto_pool ? std::min(budget, est) : (size_t)o.pool_bytes;
        if (pool_bytes < gstep)
            throw Err(BEM_ERR_NOMEM, "compression pool of " + std::to_string(pool_bytes) + " bytes cannot hold one step (" +
                                         std::to_string(gstep) + " bytes)");
    }
    const bool grouped = !gblk.empty() || gpos < nb;
    if (C->pool.bytes < pool_bytes) {
        C->pool.release();
        C->pool.alloc(pool_bytes);
    }
    BEM_HIP_TRY(hipMemsetAsync(top_dev, 0, sizeof(unsigned long long), st));
    A.pool = C->pool.as<char>();
    A.pool_cap = C->pool.bytes;
    A.sel = nullptr;
    if (grouped) {
        std::fill(selh.begin(), selh.end(), (unsigned char)0);
        for (int b : grp) selh[b] = 1;
        BEM_HIP_TRY(hipMemcpyAsync(sel_dev.p, selh.data(), (size_t)nb, hipMemcpyHostToDevice, st));
        A.sel = sel_dev.as<unsigned char>();
    }
    launch_init(A, st);
    A.sel = nullptr;
    // in-loop order: scratch slots for the ACA blocks of this group, in chunks of at most
    // ACA_SLOTS faces and the scratch buffer
    auto il_slot_doubles = [&](int b) {
        const BlockIn& Bi = C->blocks[b];
        return (aca_scratch_doubles(Bi.rs, Bi.cs, kmax, ACA_HALVES) + 31) & ~(size_t)31;
    };
    DevBuf il_scratch(&ctx->cache);
    if (iloop) {
        size_t all = 0, big = 0;
        for (int b : grp)
            if (C->blocks[b].aca) {
                all += il_slot_doubles(b);
                big = std::max(big, il_slot_doubles(b));
            }
        size_t fr = 0, tot = 0;
        BEM_HIP_TRY(hipMemGetInfo(&fr, &tot));
        const size_t budget = std::min<size_t>(ACA_SCRATCH_BYTES, (size_t)(0.25 * (double)(fr + ctx->cache.cached)));
        if (all) il_scratch.alloc(std::max(big * sizeof(double), std::min(all * sizeof(double), budget)));
    }
    std::vector<int> il_items, il_tiles, il_n0, il_t0;
    std::vector<long long> il_soff;
    std::vector<hipEvent_t> il_ev;
    // phase A: 3D-ACA of every block on dense residual faces, one step d per pass; the
    // face kernels of each step are bracketed by events (read after the next sync)
    bool face_pending = false;
    // between steps only the blocks' activity comes back: one byte per block, pinned
    DevBuf flags_dev;
    flags_dev.alloc((size_t)nb + 64);
    unsigned char* flags = nullptr;
    BEM_HIP_TRY(hipHostMalloc((void**)&flags, (size_t)nb + 64, hipHostMallocDefault));
    struct PinnedFree {
        unsigned char* p;
        ~PinnedFree() { if (p) (void)hipHostFree(p); }
    } flags_guard{flags};
    int* pending_h = (int*)(flags + (((size_t)nb + 3) & ~(size_t)3));  // in the pinned tail
    for (int d = 0; d < L; ++d) {
        launch_active_flags(A, flags_dev.as<unsigned char>(), st);
        BEM_HIP_TRY(hipMemcpyAsync(flags, flags_dev.p, (size_t)nb, hipMemcpyDeviceToHost, st));
        BEM_HIP_TRY(hipStreamSynchronize(st));
        for (int b = 0; b < nb; ++b) S[b].active = flags[b];
        if (face_pending) {
            float ms = 0.f;
            BEM_HIP_TRY(hipEventElapsedTime(&ms, evf0, evf1));
            face_ms += ms;
            face_pending = false;
        }
        ensure_pool(A, [&] {
            size_t need = 0;
            for (int b = 0; b < nb; ++b)
                if (S[b].active) need += step_bytes(b);
            return need;
        }());
        tiles.clear();
        act.clear();
        // tiles grouped by face-kernel path (one instantiation per group): regular tiles
        // of complex64 / complex128 blocks -> 1 / 2, near tiles -> 3 / 0, self tiles -> 5 / 4
        constexpr int NPATH = 6;
        size_t pstart[NPATH + 1] = {0, 0, 0, 0, 0, 0, 0};
        for (int path = 0; path < NPATH; ++path) {
            pstart[path] = tiles.size();
            for (int b = 0; b < nb; ++b) {
                const BlockIn& B = C->blocks[b];
                if (!S[b].active) continue;
                const int tn = B.ntr + (B.n1 + TILE / 4 - 1) / (TILE / 4) + (B.n2 + TILE / 16 - 1) / (TILE / 16);
                const int preg = B.f32 ? 1 : 2, pnear = B.f32 ? 3 : 0, pself = B.f32 ? 5 : 4;
                if (path == preg)
                    for (int t = 0; t < B.ntr; ++t) tiles.push_back((b << 12) | t);
                if (path == pnear)
                    for (int t = B.ntr; t < tn; ++t) tiles.push_back((b << 12) | t);
                if (path == pself)
                    for (int t = tn; t < B.ntile; ++t) tiles.push_back((b << 12) | t);
            }
        }
        pstart[NPATH] = tiles.size();
        for (int b = 0; b < nb; ++b)
            if (S[b].active) act.push_back(b);
        if (act.empty()) break;
        const int* p_tiles = put_list(list_dev, 0, tiles, st);
        const int* p_act = put_list(list_dev, tiles.size(), act, st);
        A.d = d;
        int64_t pairs = 0;
        for (int b : act) {
            const BlockIn& B = C->blocks[b];
            pairs += (int64_t)B.rs * B.cs;
            face_bytes += (double)B.rs * B.cs * 9.0 * (B.f32 ? sizeof(zf) : sizeof(zd)) * (d + 1);
        }
        face_pairs += pairs;
        face_flop += (double)pairs * (QPTS_REGULAR * flops_eval(op) + FLOPS_RESIDUAL * d);
        BEM_HIP_TRY(hipEventRecord(evf0, st));
        for (int path = 0; path < NPATH; ++path) {
            A.list = p_tiles + pstart[path];
            A.nlist = (int)(pstart[path + 1] - pstart[path]);
            if (A.nlist) ++face_launches;
            launch_face_dense(A, path, st);
        }
        BEM_HIP_TRY(hipEventRecord(evf1, st));
        face_pending = true;
        A.list = p_act;
        A.nlist = (int)act.size();
        if (d > 0) launch_final_prev(A, st);  // trace-form terms of step d - 1 came with the faces
        if (iloop) {
            // Sec. 3.1 order: the residual faces of this step's ACA blocks are approximated by
            // the ACA + recompression, and the pivot below is searched on the reconstruction
            il_items.clear();
            il_tiles.clear();
            il_soff.clear();
            il_n0.clear();
            il_t0.clear();
            size_t bytes = 0;
            for (int b : act) {
                const BlockIn& Bi = C->blocks[b];
                if (!Bi.aca) continue;
                const size_t sz = il_slot_doubles(b);
                if (il_n0.empty() || il_items.size() - (size_t)il_n0.back() >= ACA_SLOTS ||
                    (bytes + sz) * sizeof(double) > il_scratch.bytes) {
                    il_n0.push_back((int)il_items.size());
                    il_t0.push_back((int)il_tiles.size());
                    bytes = 0;
                }
                il_soff.push_back((long long)bytes);
                bytes += sz;
                il_items.push_back((b << 8) | d);
                for (int t = 0; t < Bi.ntile; ++t) il_tiles.push_back((b << 12) | t);
            }
            il_n0.push_back((int)il_items.size());
            il_t0.push_back((int)il_tiles.size());
            if (!il_items.empty()) {
                const int* p_items = put_list(il_list_dev, 0, il_items, st);
                const int* p_itiles = put_list(il_list_dev, il_items.size(), il_tiles, st);
                BEM_HIP_TRY(hipMemcpyAsync(il_slot_dev.p, il_soff.data(), il_soff.size() * sizeof(long long),
                                           hipMemcpyHostToDevice, st));
                A.scratch = il_scratch.as<double>();
                A.iloop = 1;
                for (size_t ci = 0; ci + 1 < il_n0.size(); ++ci) {
                    hipEvent_t e[4];
                    for (hipEvent_t& ev : e) {
                        BEM_HIP_TRY(hipEventCreate(&ev));
                        il_ev.push_back(ev);
                    }
                    A.list = p_items + il_n0[ci];
                    A.nlist = il_n0[ci + 1] - il_n0[ci];
                    A.slot_off = il_slot_dev.as<long long>() + il_n0[ci];
                    BEM_HIP_TRY(hipEventRecord(e[0], st));
                    launch_face_aca(A, st, 0);
                    BEM_HIP_TRY(hipEventRecord(e[1], st));
                    launch_face_recomp(A, st);
                    BEM_HIP_TRY(hipEventRecord(e[2], st));
                    launch_iloop_store(A, st);
                    A.list = p_itiles + il_t0[ci];
                    A.nlist = il_t0[ci + 1] - il_t0[ci];
                    launch_iloop_recon(A, st);
                    BEM_HIP_TRY(hipEventRecord(e[3], st));
                    ++aca_launches;
                    ++recomp_launches;
                }
                A.iloop = 0;
                A.scratch = nullptr;
                A.slot_off = nullptr;
                A.list = p_act;
                A.nlist = (int)act.size();
            }
        }
        launch_pivot(A, st);
        launch_fibre(A, st);
        launch_advance(A, st);
        A.list = p_tiles;
        A.nlist = (int)tiles.size();
        launch_cross_dense(A, st);  // blocks without a next frequency only
        A.list = p_act;
        A.nlist = (int)act.size();
        launch_final(A, st);
    }
    // dense fallback of the blocks without a regular pivot
    BEM_HIP_TRY(hipMemcpyAsync(S.data(), st_dev.p, sizeof(BlockState) * nb, hipMemcpyDeviceToHost, st));
    BEM_HIP_TRY(hipStreamSynchronize(st));
    if (face_pending) {
        float ms = 0.f;
        BEM_HIP_TRY(hipEventElapsedTime(&ms, evf0, evf1));
        face_ms += ms;
    }
    std::vector<int> fb_blocks, fb_tiles;
    for (int b : grp)
        if (S[b].fallback) {
            fb_blocks.push_back(b);
            for (int t = 0; t < C->blocks[b].ntile; ++t) fb_tiles.push_back((b << 12) | t);
        }
    if (!fb_blocks.empty()) {
        size_t need = 0;
        for (int b : fb_blocks) need += (size_t)L * step_bytes(b);
        ensure_pool(A, need);
        const int* p_fb = put_list(list_dev, 0, fb_blocks, st);
        const int* p_ft = put_list(list_dev, fb_blocks.size(), fb_tiles, st);
        for (int kf = 0; kf < L; ++kf) {
            A.list = p_fb;
            A.nlist = (int)fb_blocks.size();
            launch_fallback(A, kf, st);
            A.list = p_ft;
            A.nlist = (int)fb_tiles.size();
            launch_fallback_faces(A, kf, st);
        }
    }
    if (iloop) {
        // the faces kept as factors replace their reconstructions
        std::vector<int> ab;
        for (int b : grp)
            if (C->blocks[b].aca) ab.push_back(b);
        if (!ab.empty()) {
            A.list = put_list(il_list_dev, 0, ab, st);
            A.nlist = (int)ab.size();
            launch_iloop_finish(A, st);
        }
    }
    BEM_HIP_TRY(hipStreamSynchronize(st));
    for (size_t e = 0; e < il_ev.size(); e += 4) {
        float ms = 0.f;
        BEM_HIP_TRY(hipEventElapsedTime(&ms, il_ev[e], il_ev[e + 1]));
        aca_kernel_ms += ms;
        BEM_HIP_TRY(hipEventElapsedTime(&ms, il_ev[e + 1], il_ev[e + 2]));
        recomp_ms += ms;
        BEM_HIP_TRY(hipEventElapsedTime(&ms, il_ev[e], il_ev[e + 3]));
        aca_ms += ms;
    }
    for (hipEvent_t e : il_ev) (void)hipEventDestroy(e);
    il_ev.clear();
    BEM_HIP_TRY(hipMemcpy(&err, err_dev, sizeof(int), hipMemcpyDeviceToHost));
    if (err & 2) {
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
        (void)hipEventDestroy(ev2);
        (void)hipEventDestroy(evf0);
        (void)hipEventDestroy(evf1);
        throw Err(BEM_ERR_NOMEM, "compression pool overflowed");
    }
    BEM_HIP_TRY(hipMemcpy(S.data(), st_dev.p, sizeof(BlockState) * nb, hipMemcpyDeviceToHost));
    // phase B: per-slice ACA + recompression of the far faces of the ACA blocks, in place
    std::vector<int> items;
    for (int b : grp)
        if (C->blocks[b].aca && !S[b].fallback && !iloop)
            for (int d = 0; d < S[b].rank; ++d) items.push_back((b << 8) | d);
    // largest faces first: the long workgroups start early instead of forming the tail
    std::stable_sort(items.begin(), items.end(), [&](int x, int y) {
        const BlockIn& X = C->blocks[x >> 8];
        const BlockIn& Y = C->blocks[y >> 8];
        return (int64_t)X.rs * X.cs > (int64_t)Y.rs * Y.cs;
    });
    BEM_HIP_TRY(hipEventRecord(ev1, st));
    if (!items.empty()) {
        // scratch slots sized by each face's own dimensions, in chunks of at most ACA_SLOTS
        // faces and ACA_SCRATCH_BYTES (or a quarter of the memory when that is less): the
        // scratch buffer then has the same size in every compression of the operator and is
        // served again from the context's cache
        std::vector<long long> soff(items.size());
        std::vector<size_t> chunk0;
        size_t fr = 0, tot = 0;
        BEM_HIP_TRY(hipMemGetInfo(&fr, &tot));
        const size_t budget = std::min<size_t>(ACA_SCRATCH_BYTES, (size_t)(0.25 * (double)(fr + ctx->cache.cached)));
        size_t chunk_bytes = 0, max_bytes = 0;
        for (size_t i = 0; i < items.size(); ++i) {
            const BlockIn& Bi = C->blocks[items[i] >> 8];
            const size_t sz = (aca_scratch_doubles(Bi.rs, Bi.cs, kmax, ACA_HALVES) + 31) & ~(size_t)31;
            if (chunk0.empty() || i - chunk0.back() >= ACA_SLOTS || (chunk_bytes + sz) * sizeof(double) > budget) {
                chunk0.push_back(i);
                chunk_bytes = 0;
            }
            soff[i] = (long long)chunk_bytes;
            chunk_bytes += sz;
            max_bytes = std::max(max_bytes, chunk_bytes * sizeof(double));
        }
        chunk0.push_back(items.size());
        DevBuf scratch(&ctx->cache);
        scratch.alloc(max_bytes);
        A.scratch = scratch.as<double>();
        const int* p_items = put_list(list_dev, 0, items, st);
        DevBuf soff_dev;
        soff_dev.alloc(soff.size() * sizeof(long long));
        BEM_HIP_TRY(hipMemcpyAsync(soff_dev.p, soff.data(), soff.size() * sizeof(long long), hipMemcpyHostToDevice, st));
        std::vector<hipEvent_t> evr;
        for (size_t ci = 0; ci + 1 < chunk0.size(); ++ci) {
            const size_t c0 = chunk0[ci];
            A.list = p_items + c0;
            A.slot_off = soff_dev.as<long long>() + c0;
            A.nlist = (int)(chunk0[ci + 1] - c0);
            // first run over the chunk, then resume launches while intermediate recompressions
            // leave faces pending (the count comes back through pinned memory)
            for (int round = 0; round <= o.aca_rounds; ++round) {
                if (round > 0) {
                    BEM_HIP_TRY(hipMemcpyAsync(pending_h, A.pending, sizeof(int), hipMemcpyDeviceToHost, st));
                    BEM_HIP_TRY(hipStreamSynchronize(st));
                    if (*pending_h == 0) break;
                }
                BEM_HIP_TRY(hipMemsetAsync(A.pending, 0, sizeof(int), st));
                hipEvent_t e[3];
                for (hipEvent_t& ev : e) {
                    BEM_HIP_TRY(hipEventCreate(&ev));
                    evr.push_back(ev);
                }
                BEM_HIP_TRY(hipEventRecord(e[0], st));
                launch_face_aca(A, st, round > 0 ? 1 : 0);
                BEM_HIP_TRY(hipEventRecord(e[1], st));
                launch_face_recomp(A, st);
                BEM_HIP_TRY(hipEventRecord(e[2], st));
                ++aca_launches;
                ++recomp_launches;
            }
        }
        BEM_HIP_TRY(hipStreamSynchronize(st));
        for (size_t e = 0; e < evr.size(); e += 3) {
            float ms = 0.f;
            BEM_HIP_TRY(hipEventElapsedTime(&ms, evr[e], evr[e + 1]));
            aca_kernel_ms += ms;
            BEM_HIP_TRY(hipEventElapsedTime(&ms, evr[e + 1], evr[e + 2]));
            recomp_ms += ms;
        }
        for (hipEvent_t e : evr) (void)hipEventDestroy(e);
    }
    BEM_HIP_TRY(hipEventRecord(ev2, st));
    BEM_HIP_TRY(hipStreamSynchronize(st));
    {
        float ms = 0.f;
        BEM_HIP_TRY(hipEventElapsedTime(&kms, ev0, ev2));
        BEM_HIP_TRY(hipEventElapsedTime(&ms, ev1, ev2));
        aca_ms += ms;
    }
    BEM_HIP_TRY(hipMemcpy(S.data(), st_dev.p, sizeof(BlockState) * nb, hipMemcpyDeviceToHost));
    BEM_HIP_TRY(hipMemcpy(fh.data(), C->faces_dev.p, sizeof(FaceDesc) * (size_t)nb * L, hipMemcpyDeviceToHost));
    for (int b : grp) std::copy(fh.begin() + (size_t)b * L, fh.begin() + (size_t)(b + 1) * L, C->faces.begin() + (size_t)b * L);

    // phase C: compaction of the kept faces, factors and fibres into a pool of exact size
    {
        auto kept_bytes = [&](const FaceDesc& f, const BlockIn& B) -> long long {
            const long long zs = f.fp32 ? (long long)sizeof(zf) : (long long)sizeof(zd);
            if (f.kk == 0) return zs * 9 * B.rs * B.cs;
            if (f.kk > 0) return zs * 3 * (B.rs + B.cs) * f.kk;
            return 0;
        };
        auto up256 = [](long long v) { return (v + 255) & ~255LL; };
        std::vector<long long> seg;
        long long top = 0;
        for (int b : grp) {
            const BlockIn& B = C->blocks[b];
            for (int d = 0; d < S[b].rank; ++d) {
                FaceDesc& f = C->faces[(size_t)b * L + d];
                const long long fb = kept_bytes(f, B);
                if (fb > 0) {
                    seg.insert(seg.end(), {f.face_off, top, fb});
                    f.face_off = top;
                    top = up256(top + fb);
                }
                const long long nbf = (long long)sizeof(zd) * 9 * L;
                seg.insert(seg.end(), {f.fib_off, top, nbf});
                f.fib_off = top;
                top = up256(top + nbf);
            }
        }
        DevBuf np(&ctx->cache), segd;
        bool ok = true;
        try {
            np.alloc(std::max<long long>(top, 256), true);
            segd.alloc(std::max<size_t>(seg.size(), 3) * sizeof(long long));
        } catch (const DevBuf::bem_nomem&) {
            ok = false;  // not enough memory for the copy: keep the working pool
        }
        if (ok) {
            const int nseg = (int)(seg.size() / 3);
            if (nseg) {
                BEM_HIP_TRY(hipMemcpyAsync(segd.p, seg.data(), seg.size() * sizeof(long long), hipMemcpyHostToDevice, st));
                launch_copy_segments(C->pool.as<char>(), np.as<char>(), segd.as<long long>(), nseg, st);
            }
            BEM_HIP_TRY(hipStreamSynchronize(st));
            if (grouped) {
                gpools.push_back(std::make_unique<DevBuf>(&ctx->cache));
                gpools.back()->swap(np);
                gblk.push_back(grp);
            } else {
                C->pool.swap(np);
            }
            np.release();
        } else {
            // not enough memory for the copy: a single group keeps its working pool
            if (grouped) {
                size_t kept = 0;
                for (const auto& g : gpools) kept += g->bytes;
                throw Err(BEM_ERR_NOMEM, "device memory exhausted by the compaction of block group " +
                                             std::to_string(gpools.size()) + " (" + std::to_string(top) +
                                             " bytes; earlier groups hold " + std::to_string(kept) +
                                             " bytes, the working pool " + std::to_string(C->pool.bytes) + ")");
            }
            for (int b : grp)
                std::copy(fh.begin() + (size_t)b * L, fh.begin() + (size_t)(b + 1) * L, C->faces.begin() + (size_t)b * L);
        }
    }
    }  // block groups
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    (void)hipEventDestroy(ev2);
    (void)hipEventDestroy(evf0);
    (void)hipEventDestroy(evf1);
    if (!gpools.empty()) {
        // the operator's pool is the group pool at the lowest address; the faces of every
        // group are addressed from its base
        C->pool.release();
        size_t lo = 0;
        for (size_t g = 1; g < gpools.size(); ++g)
            if ((uintptr_t)gpools[g]->p < (uintptr_t)gpools[lo]->p) lo = g;
        const uintptr_t base = (uintptr_t)gpools[lo]->p;
        for (size_t g = 0; g < gpools.size(); ++g) {
            const long long delta = (long long)((uintptr_t)gpools[g]->p - base);
            for (int b : gblk[g])
                for (int d = 0; d < S[b].rank; ++d) {
                    FaceDesc& f = C->faces[(size_t)b * L + d];
                    f.face_off += delta;
                    f.fib_off += delta;
                }
        }
        C->pool.swap(*gpools[lo]);
        for (size_t g = 0; g < gpools.size(); ++g)
            if (g != lo) C->extra_pools.push_back(std::move(gpools[g]));
        C->ngroups_c = (int)gpools.size();
    }
    C->faces_dev.release();
    build_apply_plan(*C, st);
    build_mplan(*C, st);

    // statistics
    bem_stats& R = out->stats;
    std::memset(&R, 0, sizeof(R));
    R.n_blocks = nb;
    R.n_far = n_far;
    R.n_near = nb - n_far;
    R.rank_min = L + 1;
    double rsum = 0, acasum = 0, colsum = 0, rflop = 0;
    int64_t nfarfaces = 0, bytes = 0, ent = 0;
    for (int b = 0; b < nb; ++b) {
        const BlockState& s = S[b];
        const BlockIn& B = C->blocks[b];
        R.n_dense_fallback += s.fallback;
        R.rank_min = std::min(R.rank_min, s.rank);
        R.rank_max = std::max(R.rank_max, s.rank);
        rsum += s.rank;
        ent += s.entries;
        R.entries_regular += (int64_t)s.rank * B.nreg;
        R.entries_near += (int64_t)s.rank * (B.n1 + B.n2);
        R.entries_self += (int64_t)s.rank * B.n3;
        R.n_aca_dense += s.aca_dense;
        colsum += (double)s.aca_cols;
        rflop += s.recomp_flop;
        R.aca_flop += s.aca_flop;
        R.aca_bytes += s.aca_bytes;
        for (int d = 0; d < s.rank; ++d) {
            const FaceDesc& f = C->faces[(size_t)b * L + d];
            bytes += (int64_t)L * 9 * sizeof(zd);
            size_t zs = f.fp32 ? sizeof(zf) : sizeof(zd);
            if (f.kk >= 0) {
                const double core = f.kk > 0 ? 3.0 * (B.rs + B.cs) * f.kk : 9.0 * B.rs * B.cs;
                if (f.sel) R.apply_macs_sel += core;
                else (f.fp32 ? R.apply_macs_c64 : R.apply_macs_c128) += core;
                if (!f.sel) R.apply_macs_fibre += 9.0 * B.cs;
            }
            if (f.kk == 0) {
                bytes += (int64_t)9 * B.rs * B.cs * (int64_t)zs;
            } else if (f.kk > 0) {
                bytes += (int64_t)3 * (B.rs + B.cs) * f.kk * (int64_t)zs;
                acasum += f.kk;
                ++nfarfaces;
                R.aca_rank_max = std::max(R.aca_rank_max, f.kk);
            }
        }
    }
    R.rank_mean = nb ? rsum / nb : 0.0;
    R.aca_rank_mean = nfarfaces ? acasum / nfarfaces : 0.0;
    R.aca_cols_mean = nfarfaces ? colsum / nfarfaces : 0.0;
    R.bytes = bytes;
    {
        // dense size: the M x M x L array of each component (one for a single mesh)
        double dense = 0.0;
        if (ctx->hgeo.ncomp > 1) {
            std::vector<double> kc(ctx->hgeo.ncomp, 0.0);
            for (int c : ctx->hgeo.comp) kc[c] += 1.0;
            for (double k : kc) dense += (double)L * 9.0 * k * k * 16.0;
        } else {
            dense = (double)L * 9.0 * (double)K * (double)K * 16.0;
        }
        R.compression_rate = (double)bytes / dense;
    }
    R.entries_generated = ent;
    R.entries_other = ent - R.entries_regular - R.entries_near - R.entries_self;
    R.n_far_faces = nfarfaces;
    R.kernel_ms = kms;
    R.aca_ms = aca_ms;
    R.face_ms = face_ms;
    R.face_launches = face_launches;
    R.face_pairs = face_pairs;
    R.face_flop = face_flop;
    R.face_bytes = face_bytes;
    R.block_groups = C->ngroups_c;
    R.recomp_ms = recomp_ms;
    R.recomp_launches = recomp_launches;
    R.aca_kernel_ms = aca_kernel_ms;
    R.aca_launches = aca_launches;
    R.recomp_flop = rflop;
    R.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return BEM_OK;
}

void aca_matrix_impl(bem_ctx* ctx, bool fp32, int m, int n, const void* A, double tol, int max_cols, int* kc, int* kk,
                     void* U, void* V)
{
    hipStream_t st = ctx->stream;
    int cap = max_cols > 0 ? max_cols : face_aca_cap(m, n);
    cap = std::min({cap, 3 * std::min(m, n), KMAX_ACA});
    cap -= cap % 3;
    const int kmax = std::max(cap, 3);
    const size_t zs = fp32 ? sizeof(zf) : sizeof(zd);
    const size_t bytes = zs * 9 * (size_t)m * n;
    DevBuf h, scratch, out;
    h.alloc(bytes);
    scratch.alloc(((aca_scratch_doubles(m, n, kmax) + 31) & ~(size_t)31) * sizeof(double));
    out.alloc(64);
    BEM_HIP_TRY(hipMemcpyAsync(h.p, A, bytes, hipMemcpyHostToDevice, st));
    launch_aca_matrix(h.as<char>(), m, n, fp32 ? 1 : 0, tol, cap, kmax, scratch.as<double>(), out.as<int>(), st);
    int r[2] = {0, 0};
    BEM_HIP_TRY(hipMemcpyAsync(r, out.p, sizeof(r), hipMemcpyDeviceToHost, st));
    BEM_HIP_TRY(hipStreamSynchronize(st));
    *kc = r[0];
    *kk = r[1];
    if (r[1] > 0) {
        const size_t ub = zs * 3 * (size_t)m * r[1], vb = zs * 3 * (size_t)n * r[1];
        if (U) BEM_HIP_TRY(hipMemcpy(U, h.p, ub, hipMemcpyDeviceToHost));
        if (V) BEM_HIP_TRY(hipMemcpy(V, h.as<char>() + ub, vb, hipMemcpyDeviceToHost));
    }
}

void apply_compressed(bem_op* op, int nrhs, const zd* x_dev, int64_t x_l_stride, zd* y_dev, hipStream_t st)
{
    CompressedOp& C = *op->comp;
    const size_t M = 3 * (size_t)C.K;
    const size_t ncols = (size_t)C.L * nrhs;
    const MPlan::Segs& S = (ncols + MFMA_COLS - 1) / MFMA_COLS <= 2 ? C.mp.fine : C.mp.coarse;
    const size_t prow = (size_t)3 * MFMA_ROW_CHUNK * ncols;  // partial rows of one segment
    size_t need = (2 * ncols * M + (size_t)C.far_rows * ncols + (size_t)S.nseg * prow + 16) * sizeof(zd);
    if (C.work.bytes < need) C.work.alloc(need);
    zd* xp = C.work.as<zd>();
    zd* yp = xp + ncols * M;
    zd* tb = yp + ncols * M;
    launch_permute(x_dev, xp, C.perm_dev.as<int>(), C.K, C.L, nrhs, x_l_stride, true, st);
    MApplyArgs A = margs(C.mp, S, C.blocks_dev, C.af_dev, C.pool.as<char>(), C.K, C.L, nrhs);
    A.x = xp;
    A.y = yp;
    A.tbuf = tb;
    A.pbuf = tb + (size_t)C.far_rows * ncols;
    launch_apply_mfma(A, st);
    launch_permute(yp, y_dev, C.perm_dev.as<int>(), C.K, C.L, nrhs, (int64_t)M, false, st);
}

// Plan of the transposed product: the same chunks (the partition is square), each with the
// faces of the blocks whose columns cover it.
void build_apply_plan_t(CompressedOp& C, hipStream_t st)
{
    const int nb = (int)C.blocks.size();
    std::vector<std::vector<int>> faces_of_block(nb);
    for (size_t f = 0; f < C.af.size(); ++f) faces_of_block[C.af[f].block].push_back((int)f);
    const std::vector<int>& s2 = C.h_start;
    std::vector<std::vector<int>> lists(C.ngroups);
    for (int b = 0; b < nb; ++b) {
        const BlockIn& B = C.blocks[b];
        auto it = std::lower_bound(s2.begin(), s2.end(), B.cb);
        for (; it != s2.end() && *it < B.cb + B.cs; ++it)
            for (int fi : faces_of_block[b]) lists[it - s2.begin()].push_back(fi);
    }
    std::vector<int> ptr(C.ngroups + 1, 0), flat;
    for (int g = 0; g < C.ngroups; ++g) {
        ptr[g + 1] = ptr[g] + (int)lists[g].size();
        flat.insert(flat.end(), lists[g].begin(), lists[g].end());
    }
    std::vector<int> segbuf = make_segments(C.af, C.blocks, ptr, flat, APPLY_SEGMENTS, &C.nseg_t, true);
    auto up = [&](DevBuf& d, const void* src, size_t bytes) {
        d.alloc(std::max<size_t>(bytes, 16));
        if (bytes) BEM_HIP_TRY(hipMemcpyAsync(d.p, src, bytes, hipMemcpyHostToDevice, st));
    };
    up(C.rowfaces_t_dev, flat.data(), flat.size() * sizeof(int));
    up(C.rowptr_t_dev, ptr.data(), ptr.size() * sizeof(int));
    up(C.seg_t_dev, segbuf.data(), segbuf.size() * sizeof(int));
    BEM_HIP_TRY(hipStreamSynchronize(st));
    C.t_built = true;
}

void apply_compressed_t(bem_op* op, int nrhs, const zd* x_dev, zd* y_dev, hipStream_t st)
{
    CompressedOp& C = *op->comp;
    if (!C.t_built) build_apply_plan_t(C, st);
    const size_t M = 3 * (size_t)C.K;
    const size_t ncols = (size_t)C.L * nrhs;
    const size_t prow = (size_t)3 * APPLY_ROW_CHUNK * ncols;
    size_t need = (2 * ncols * M + (size_t)C.far_rows * ncols + (size_t)C.nseg_t * prow + 16) * sizeof(zd);
    if (C.work.bytes < need) C.work.alloc(need);
    zd* xp = C.work.as<zd>();
    zd* yp = xp + ncols * M;
    zd* tb = yp + ncols * M;
    launch_permute(x_dev, xp, C.perm_dev.as<int>(), C.K, C.L, nrhs, (int64_t)M, true, st);
    ApplyArgs A = plan_args(C, nrhs);
    A.row_faces = C.rowfaces_t_dev.as<int>();
    A.row_ptr = C.rowptr_t_dev.as<int>();
    A.nseg = C.nseg_t;
    A.seg_group = C.seg_t_dev.as<int>();
    A.seg_begin = A.seg_group + C.nseg_t;
    A.group_seg = A.seg_begin + C.nseg_t + 1;
    A.x = xp;
    A.y = yp;
    A.tbuf = tb;
    A.pbuf = tb + (size_t)C.far_rows * ncols;
    launch_apply_t(A, st);
    launch_permute(yp, y_dev, C.perm_dev.as<int>(), C.K, C.L, nrhs, (int64_t)M, false, st);
}

void apply_weighted_compressed(bem_op* op, const zd* W_dev, zd* y_dev, hipStream_t st)
{
    CompressedOp& C = *op->comp;
    const size_t M = 3 * (size_t)C.K;
    const size_t prow = (size_t)3 * APPLY_ROW_CHUNK;
    size_t need = ((size_t)C.L * M + M + (size_t)C.zw_total + (size_t)C.far_rows + (size_t)std::max(C.nseg, C.nsegf) * prow + 16) *
                  sizeof(zd);
    if (C.work.bytes < need) C.work.alloc(need);
    zd* Wp = C.work.as<zd>();
    zd* yp = Wp + (size_t)C.L * M;
    zd* zw = yp + M;
    zd* tb = zw + C.zw_total;
    launch_permute(W_dev, Wp, C.perm_dev.as<int>(), C.K, C.L, 1, (int64_t)M, true, st);
    ApplyArgs A = plan_args(C, 1);
    A.x = Wp;
    A.y = yp;
    A.tbuf = tb;
    A.pbuf = tb + C.far_rows;
    launch_weighted(A, Wp, zw, yp, st);
    launch_permute(yp, y_dev, C.perm_dev.as<int>(), C.K, 1, 1, (int64_t)M, false, st);
}

void apply_sum_compressed(bem_op* op, const zd* x_dev, double scale, zd* y_dev, hipStream_t st)
{
    CompressedOp& C = *op->comp;
    const size_t M = 3 * (size_t)C.K;
    const size_t prow = (size_t)3 * APPLY_ROW_CHUNK;
    size_t need = (2 * M + (size_t)C.zw_total + (size_t)C.far_rows + (size_t)std::max(C.nseg, C.nsegf) * prow + 16) *
                  sizeof(zd);
    if (C.work.bytes < need) C.work.alloc(need);
    zd* xp = C.work.as<zd>();
    zd* yp = xp + M;
    zd* zw = yp + M;
    zd* tb = zw + C.zw_total;
    launch_permute(x_dev, xp, C.perm_dev.as<int>(), C.K, 1, 1, (int64_t)M, true, st);
    ApplyArgs A = plan_args(C, 1);
    A.x = xp;
    A.y = yp;
    A.tbuf = tb;
    A.pbuf = tb + C.far_rows;
    launch_weighted(A, xp, zw, yp, st, true, scale);
    launch_permute(yp, y_dev, C.perm_dev.as<int>(), C.K, 1, 1, (int64_t)M, false, st);
}

void compressed_blocks(const bem_op* op, int64_t* n, int64_t* rows, int32_t* perm)
{
    const CompressedOp& C = *op->comp;
    *n = (int64_t)C.blocks.size();
    if (rows)
        for (size_t b = 0; b < C.blocks.size(); ++b) {
            const BlockIn& B = C.blocks[b];
            int64_t cols = 0;
            for (int d = 0; d < C.st[b].rank; ++d) cols += std::max(0, C.faces[b * C.L + d].kk);
            int64_t r[8] = {B.rb, B.rs, B.cb, B.cs, B.far, C.st[b].rank, C.st[b].fallback, cols};
            std::memcpy(rows + 8 * b, r, sizeof(r));
        }
    if (perm)
        for (int e = 0; e < C.K; ++e) perm[e] = C.part.perm[e];
}

void compressed_freq_hist(const bem_op* op, int64_t* hist)
{
    const CompressedOp& C = *op->comp;
    for (int l = 0; l < C.L; ++l) hist[l] = 0;
    for (size_t b = 0; b < C.blocks.size(); ++b) {
        if (C.st[b].fallback) continue;
        for (int d = 0; d < C.st[b].rank; ++d) hist[C.faces[b * C.L + d].k]++;
    }
}


// ---------------------------------------------------------------- batched products

struct BatchPlan {
    std::vector<bem_op*> ops;
    int nrhs = 0, L = 0, Ktot = 0, Kmax = 0;
    std::vector<int> koff;
    // merged plan (host): blocks, faces and the chunks of the product on the matrix cores
    std::vector<BlockIn> blocks;
    std::vector<ApplyFace> af;
    MPlan mp;
    long long far_rows = 0;
    const char* base = nullptr;
    DevBuf blocks_dev, af_dev, far_sorted_dev;
    // schedule
    int seg_target = 0, far_sorted = 0;
    std::vector<double> tune_ms;
    std::vector<int> tune_seg;
    DevBuf work;
    size_t work_bytes = 0;
    // graph of the last device-pointer call
    bool use_graph = false;
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const void*> gx;
    std::vector<void*> gy;
    hipStream_t gstream = nullptr;
    int graph_builds = 0, graph_launches = 0;
    double flop = 0.0;  // algorithmic flops of one product
    ~BatchPlan()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

namespace {

size_t batch_work_bytes(const BatchPlan& P, int nseg)
{
    const size_t ncols = (size_t)P.L * P.nrhs, M = 3 * (size_t)P.Ktot;
    return (2 * ncols * M + (size_t)P.far_rows * ncols + (size_t)nseg * 3 * MFMA_ROW_CHUNK * ncols + 16) * sizeof(zd);
}

void batch_set_segments(BatchPlan& P, int target, hipStream_t st)
{
    set_msegments(P.mp.fine, P.af, P.blocks, P.mp, target, st);
    BEM_HIP_TRY(hipStreamSynchronize(st));
    P.seg_target = target;
}

MApplyArgs batch_args(const BatchPlan& P)
{
    MApplyArgs A = margs(P.mp, P.mp.fine, P.blocks_dev, P.af_dev, P.base, P.Ktot, P.L, P.nrhs);
    if (P.far_sorted) {
        A.far64 = P.far_sorted_dev.as<int>();
        A.far32 = A.far64 + P.mp.far64.size();
    }
    const size_t ncols = (size_t)P.L * P.nrhs, M = 3 * (size_t)P.Ktot;
    zd* xp = P.work.as<zd>();
    A.x = xp;
    A.y = xp + ncols * M;
    A.tbuf = xp + 2 * ncols * M;
    A.pbuf = A.tbuf + (size_t)P.far_rows * ncols;
    return A;
}

// the products of the batch: permutation in, far products, rows, row sums, permutation out
void batch_enqueue(const BatchPlan& P, const zd* const* x, zd* const* y, hipStream_t st)
{
    BatchPermTable T{};
    T.nops = (int)P.ops.size();
    T.L = P.L;
    T.nrhs = P.nrhs;
    T.Ktot = P.Ktot;
    for (int o = 0; o < T.nops; ++o) {
        const CompressedOp& C = *P.ops[o]->comp;
        T.op[o] = BatchPerm{x ? x[o] : nullptr, y ? y[o] : nullptr, C.perm_dev.as<int>(), C.K, P.koff[o]};
    }
    MApplyArgs A = batch_args(P);
    launch_permute_batch(T, P.Kmax, P.work.as<zd>(), true, st);
    launch_apply_mfma(A, st);
    launch_permute_batch(T, P.Kmax, const_cast<zd*>(A.y), false, st);
}

// Time of the products of one schedule candidate, taken on at most 512 columns (the same
// right-hand-side count in every candidate): each column tile costs the same, so the
// ranking holds for more columns while the tuner stays cheap.
double batch_time_ms(const BatchPlan& P, hipStream_t st, int reps)
{
    hipEvent_t e0, e1;
    BEM_HIP_TRY(hipEventCreate(&e0));
    BEM_HIP_TRY(hipEventCreate(&e1));
    MApplyArgs A = batch_args(P);
    A.nrhs = std::max(1, std::min(P.nrhs, 512 / P.L));
    const size_t ncols = (size_t)P.L * A.nrhs, M = 3 * (size_t)P.Ktot;
    A.y = const_cast<zd*>(A.x) + ncols * M;
    A.tbuf = const_cast<zd*>(A.x) + 2 * ncols * M;
    A.pbuf = A.tbuf + (size_t)P.far_rows * ncols;
    launch_apply_mfma(A, st);  // warm-up
    BEM_HIP_TRY(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) launch_apply_mfma(A, st);
    BEM_HIP_TRY(hipEventRecord(e1, st));
    BEM_HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    BEM_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms / reps;
}

int count_msegments(const BatchPlan& P, int target)
{
    int ns = 0, n64 = 0, n32 = 0;
    (void)make_msegments(P.af, P.blocks, P.mp.ptr, P.mp.nf64, P.mp.flat, target, &ns, &n64, &n32);
    return ns;
}

}  // namespace

BatchPlan* batch_create(bem_op* const* ops, int nops, int nrhs, int flags, hipStream_t st)
{
    auto P = std::make_unique<BatchPlan>();
    P->ops.assign(ops, ops + nops);
    P->nrhs = nrhs;
    P->L = ops[0]->L;
    P->use_graph = (flags & BEM_BATCH_GRAPH) != 0;
    // merged plan: blocks, faces, chunks and far faces of every operator, element indices
    // shifted by the operator's offset, face offsets taken from the lowest pool
    uintptr_t lo = UINTPTR_MAX;
    for (bem_op* op : P->ops) lo = std::min(lo, (uintptr_t)op->comp->pool.p);
    P->base = (const char*)lo;
    long long trow = 0;
    MPlan& mp = P->mp;
    mp.ptr.assign(1, 0);
    for (int o = 0; o < nops; ++o) {
        const CompressedOp& C = *ops[o]->comp;
        const int boff = (int)P->blocks.size(), foff = (int)P->af.size(), koff = P->Ktot;
        const long long delta = (long long)((uintptr_t)C.pool.p - lo);
        P->koff.push_back(koff);
        for (BlockIn B : C.blocks) {
            B.rb += koff;
            B.cb += koff;
            P->blocks.push_back(B);
        }
        for (ApplyFace a : C.af) {
            a.face_off += delta;
            a.fib_off += delta;
            a.block += boff;
            a.t_off += trow;
            a.zw_off = 0;
            P->af.push_back(a);
        }
        const int e0 = (int)mp.flat.size();
        for (int fi : C.mp.flat) mp.flat.push_back(fi + foff);
        for (size_t g = 1; g < C.mp.ptr.size(); ++g) mp.ptr.push_back(C.mp.ptr[g] + e0);
        mp.nf64.insert(mp.nf64.end(), C.mp.nf64.begin(), C.mp.nf64.end());
        for (int s0 : C.mp.start) mp.start.push_back(s0 + koff);
        mp.size.insert(mp.size.end(), C.mp.size.begin(), C.mp.size.end());
        for (int f : C.mp.far64) mp.far64.push_back(f + foff);
        for (int f : C.mp.far32) mp.far32.push_back(f + foff);
        trow += C.far_rows;
        P->Ktot += C.K;
        P->Kmax = std::max(P->Kmax, C.K);
    }
    mp.ngroups = (int)mp.start.size();
    P->far_rows = trow;
    // algorithmic flops of one product: per column, 9 m n complex multiply-adds for a dense
    // face, 3 (m + n) kk for factors, 9 n for the fibre (a selector face: one frequency, no
    // fibre); 8 flops each
    double macs_col = 0.0, macs_sel = 0.0;
    for (const ApplyFace& a : P->af) {
        const BlockIn& B = P->blocks[a.block];
        const double core = a.kk > 0 ? 3.0 * (B.rs + B.cs) * a.kk : 9.0 * B.rs * B.cs;
        if (a.sel) macs_sel += core;
        else macs_col += core + 9.0 * B.cs;
    }
    P->flop = 8.0 * ((double)P->L * nrhs * macs_col + (double)nrhs * macs_sel);
    std::vector<int> far = mp.far64, far_sorted;
    far.insert(far.end(), mp.far32.begin(), mp.far32.end());
    for (const std::vector<int>* lst : {&mp.far64, &mp.far32}) {
        std::vector<int> v = *lst;
        std::stable_sort(v.begin(), v.end(), [&](int a, int b) { return P->af[a].kk > P->af[b].kk; });
        far_sorted.insert(far_sorted.end(), v.begin(), v.end());
    }
    auto up = [&](DevBuf& d, const void* src, size_t bytes) {
        d.alloc(std::max<size_t>(bytes, 16));
        if (bytes) BEM_HIP_TRY(hipMemcpyAsync(d.p, src, bytes, hipMemcpyHostToDevice, st));
    };
    up(P->blocks_dev, P->blocks.data(), P->blocks.size() * sizeof(BlockIn));
    up(P->af_dev, P->af.data(), P->af.size() * sizeof(ApplyFace));
    upload_ints(mp.flat_dev, mp.flat, st);
    upload_ints(mp.start_dev, mp.start, st);
    upload_ints(mp.size_dev, mp.size, st);
    upload_ints(mp.far_dev, far, st);
    upload_ints(P->far_sorted_dev, far_sorted, st);
    // schedule: segment count and far faces in plan order or by decreasing rank; the default
    // is the single-operator schedule, the tuner times the candidates that fit in half of the
    // free memory and keeps the fastest
    const int ctiles = (P->L * nrhs + MFMA_COLS - 1) / MFMA_COLS;
    const int ng = mp.ngroups;
    const int tdef = ctiles <= 2 ? MFMA_SEGMENTS : std::max(ng, 256);
    std::vector<int> targets = {std::max(1, ng / 2), ng, 2 * ng, 4 * ng, tdef};
    std::sort(targets.begin(), targets.end());
    targets.erase(std::unique(targets.begin(), targets.end()), targets.end());
    size_t free_b = 0, total_b = 0;
    BEM_HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    std::vector<int> fit;
    for (int t : targets)
        if (batch_work_bytes(*P, count_msegments(*P, t)) <= free_b / 2 || t == targets.front()) fit.push_back(t);
    int best_t = std::find(fit.begin(), fit.end(), tdef) != fit.end() ? tdef : fit.front();
    size_t need = 0;
    if (flags & BEM_BATCH_TUNE) {
        for (int t : fit) need = std::max(need, batch_work_bytes(*P, count_msegments(*P, t)));
    } else {
        need = batch_work_bytes(*P, count_msegments(*P, best_t));
    }
    P->work.alloc(need);
    P->work_bytes = need;
    BEM_HIP_TRY(hipMemsetAsync(P->work.p, 0, need, st));
    if (flags & BEM_BATCH_TUNE) {
        double best = 1e300;
        std::vector<int> seen;
        for (int t : fit) {
            const int ns = count_msegments(*P, t);
            if (std::find(seen.begin(), seen.end(), ns) != seen.end()) continue;  // same schedule
            seen.push_back(ns);
            batch_set_segments(*P, t, st);
            const double ms = batch_time_ms(*P, st, 1);
            P->tune_seg.push_back(P->mp.fine.nseg);
            P->tune_ms.push_back(ms);
            if (ms < best) {
                best = ms;
                best_t = t;
            }
        }
        batch_set_segments(*P, best_t, st);
        P->far_sorted = 1;
        const double ms = batch_time_ms(*P, st, 1);
        P->tune_seg.push_back(P->mp.fine.nseg);
        P->tune_ms.push_back(ms);
        if (!(ms < best)) P->far_sorted = 0;
    } else {
        batch_set_segments(*P, best_t, st);
    }
    BEM_HIP_TRY(hipStreamSynchronize(st));
    return P.release();
}

void batch_apply(BatchPlan* P, const zd* const* x, zd* const* y, hipStream_t st)
{
    if (!P->use_graph) {
        batch_enqueue(*P, x, y, st);
        return;
    }
    const int n = (int)P->ops.size();
    bool same = P->exec && P->gstream == st;
    for (int o = 0; same && o < n; ++o) same = P->gx[o] == x[o] && P->gy[o] == y[o];
    if (!same) {
        if (P->exec) {
            BEM_HIP_TRY(hipGraphExecDestroy(P->exec));
            P->exec = nullptr;
        }
        if (!P->cap) BEM_HIP_TRY(hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        BEM_HIP_TRY(hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal));
        try {
            batch_enqueue(*P, x, y, P->cap);
        } catch (...) {
            (void)hipStreamEndCapture(P->cap, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        BEM_HIP_TRY(hipStreamEndCapture(P->cap, &g));
        const hipError_t e = hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        BEM_HIP_TRY(e);
        P->gx.assign(x, x + n);
        P->gy.assign(y, y + n);
        P->gstream = st;
        ++P->graph_builds;
    }
    BEM_HIP_TRY(hipGraphLaunch(P->exec, st));
    ++P->graph_launches;
}

void batch_info(const BatchPlan* P, bem_batch_info* I)
{
    *I = bem_batch_info{};
    I->nops = (int32_t)P->ops.size();
    I->nrhs = P->nrhs;
    I->L = P->L;
    I->K_total = P->Ktot;
    I->n_groups = P->mp.ngroups;
    I->n_segments = P->mp.fine.nseg;
    I->n_far_faces = (int32_t)(P->mp.far64.size() + P->mp.far32.size());
    I->seg_target = P->seg_target;
    I->persistent = 0;
    I->persistent_wgs = 0;
    I->far_sorted = P->far_sorted;
    I->graph = P->use_graph;
    I->graph_builds = P->graph_builds;
    I->graph_launches = P->graph_launches;
    I->n_tuned = (int32_t)std::min<size_t>(P->tune_ms.size(), 8);
    for (int i = 0; i < I->n_tuned; ++i) {
        I->tune_ms[i] = P->tune_ms[i];
        I->tune_segments[i] = P->tune_seg[i];
    }
    I->workspace_bytes = (double)P->work_bytes;
    I->flop = P->flop;
}

void batch_destroy(BatchPlan* P) { delete P; }

}  // namespace bem
