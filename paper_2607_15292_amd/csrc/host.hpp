// host.hpp -- host-side state of a context and an operator (shared by api.cpp,
// partition.cpp and compress.cpp).
#pragma once

#include <iterator>
#include <map>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/bem.h"
#include "lib.hpp"

namespace bem {

// Error with a BEM_ERR_* code, thrown by host code and turned into the return value at the
// C-ABI boundary.
struct ApiError : std::runtime_error {
    int code;
    ApiError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// Large device buffers released by the operators of a context are kept here and handed
// out again to allocations of similar size: repeated compressions do not return tens of
// GB to the driver and map them again.  Not thread-safe (a context is not).
struct MemCache {
    static constexpr size_t MIN_BYTES = (size_t)64 << 20;  // smaller buffers bypass the cache
    std::multimap<size_t, void*> bufs;
    size_t cached = 0;
    // smallest cached buffer of at least n bytes and at most slack * n + 64 MiB (any size when
    // slack <= 0); null if none
    void* take(size_t n, size_t* got, double slack = 1.5)
    {
        auto it = bufs.lower_bound(n);
        if (it == bufs.end() || (slack > 0 && (double)it->first > slack * (double)n + (double)(64 << 20))) return nullptr;
        void* q = it->second;
        *got = it->first;
        cached -= it->first;
        bufs.erase(it);
        return q;
    }
    void put(void* q, size_t n)
    {
        bufs.emplace(n, q);
        cached += n;
    }
    void clear()
    {
        for (auto& b : bufs) (void)hipFree(b.second);
        bufs.clear();
        cached = 0;
    }
    ~MemCache() { clear(); }
};

// Owning device allocation (through the context's MemCache when `cache` is set).
struct DevBuf {
    static constexpr size_t RESERVE = (size_t)2 << 30;  // device memory never taken (bytes)
    void* p = nullptr;
    size_t bytes = 0;
    MemCache* cache = nullptr;
    DevBuf() = default;
    explicit DevBuf(MemCache* c) : cache(c) {}
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    // lasting: the buffer outlives the call (an operator's compacted storage): a cached buffer
    // serves it only when at most 1/16 larger, never a larger one taken to save a mapping
    void alloc(size_t n, bool lasting = false)
    {
        release();
        if (n == 0) return;
        if (cache && n >= MemCache::MIN_BYTES) {
            size_t got = 0;
            if (void* q = cache->take(n, &got, lasting ? 1.0625 : 1.5)) {
                p = q;
                bytes = got;
                return;
            }
        }
        if (n >= MemCache::MIN_BYTES) {
            // leave RESERVE bytes free for the runtime (the scratch memory it allocates when
            // a kernel with a private segment starts, queues): evict cached buffers, largest
            // first, else refuse
            size_t fr = 0, tot = 0;
            if (cache && !lasting && hipMemGetInfo(&fr, &tot) == hipSuccess && fr < n + RESERVE) {
                // short of memory: a larger cached buffer serves a working buffer before any
                // is returned to the driver (freeing and mapping tens of GB takes longer than
                // the kernels)
                size_t got = 0;
                if (void* q = cache->take(n, &got, 0.0)) {
                    p = q;
                    bytes = got;
                    return;
                }
            }
            while (hipMemGetInfo(&fr, &tot) == hipSuccess && fr < n + RESERVE) {
                if (!cache || cache->bufs.empty()) throw bem_nomem(n);
                auto it = std::prev(cache->bufs.end());
                (void)hipFree(it->second);
                cache->cached -= it->first;
                cache->bufs.erase(it);
            }
        }
        hipError_t e = hipMalloc(&p, n);
        while (e != hipSuccess && cache && !cache->bufs.empty()) {  // evict, largest first
            (void)hipGetLastError();
            auto it = std::prev(cache->bufs.end());
            (void)hipFree(it->second);
            cache->cached -= it->first;
            cache->bufs.erase(it);
            e = hipMalloc(&p, n);
        }
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            throw bem_nomem(n);
        }
        bytes = n;
    }
    void release()
    {
        if (p) {
            if (cache && bytes >= MemCache::MIN_BYTES) cache->put(p, bytes);
            else (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
    }
    template <typename T> T* as() const { return (T*)p; }
    void swap(DevBuf& o)
    {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
        std::swap(cache, o.cache);
    }
    struct bem_nomem : std::runtime_error {
        explicit bem_nomem(size_t n) : std::runtime_error("device allocation of " + std::to_string(n) + " bytes failed") {}
    };
};

// Host copy of the element tables (structure of arrays, FP64).
struct HostGeo {
    int K = 0;
    std::vector<double> cx, cy, cz, nx, ny, nz, area, lmax2, vx, vy, vz, gx, gy, gz, gw;
    std::vector<int> comp;  // component of each element (empty: one component); blocks never
                            // couple two components
    int ncomp = 1;
};

// Geometry tables uploaded to the device in one allocation.
struct DevGeo {
    DevBuf buf;
    Geo geo{};
    void upload(const HostGeo& h, const int* perm /* cluster pos -> mesh elem, or null */, hipStream_t st);
};

// Cluster tree node and block of the H-matrix partition (cluster order indices).
struct Cluster {
    int begin, size;
    int child[2];
    double bmin[3], bmax[3];  // box of the element vertices
    int comp;                 // the component of all its elements, -1 when it spans several
};

struct BlockDesc {
    int rb, rs, cb, cs;  // row begin/size, column begin/size (elements, cluster order)
    int far;
};

struct Partition {
    std::vector<int> perm;        // cluster position -> mesh element
    std::vector<Cluster> nodes;   // node 0 = root
    std::vector<BlockDesc> blocks;
};

void build_partition(const HostGeo& g, double eta, int leaf, Partition& out);

struct CompressedOp;  // compress.cpp

}  // namespace bem

struct bem_ctx {
    int device = -1;
    hipStream_t stream = nullptr;
    std::string err;
    // mesh
    bool mesh_set = false;
    std::vector<double> nodes;
    std::vector<int32_t> tris;
    bem::DevBuf tris_dev;  // tris on the device (linear basis), uploaded on first use
    bem::HostGeo hgeo;
    bem::DevGeo dgeo;
    // material
    bool mat_set = false;
    double rho = 1, cp = 1, cs = 0.5;
    // frequencies
    bool freq_set = false;
    std::vector<zd> s;
    bem::DevBuf fbuf;
    bem::Freq freq{};
    // quadrature
    bem_quad quad{0, 1.5, 3.0, 8, 8};
    bem::QuadTab qtab{};
    const zd* table = nullptr;
    int live_ops = 0;
    bem::MemCache cache;  // large buffers of destroyed operators (freed with the context)

    bem::DevCtx devctx(const bem::Geo& g, const int* perm) const;
};

struct bem_op {
    bem_ctx* ctx = nullptr;
    int op = 0, prec = 0;
    int kind = 0;  // 0 dense, 1 compressed, 2 matrix-free (entries recomputed at each product)
    int K = 0, L = 0;
    bem::DevBuf dense;                               // kind 0: [L][3K][3K]
    bem::CompressedOp* comp = nullptr;               // kind 1 (owned)
    bem_stats stats{};
    int batches = 0;  // live batches that reference this operator
    ~bem_op();
};

namespace bem {
int compress_impl(bem_ctx* ctx, int op, const bem_aca_opts& o, bem_op* out);
void aca_matrix_impl(bem_ctx* ctx, bool fp32, int m, int n, const void* A, double tol, int max_cols, int* kc, int* kk,
                     void* U, void* V);
// bem_aca_matrix on device buffers with the library's static device scratch (noalloc.hip)
char* noalloc_scratch(int device);
void aca_matrix_noalloc_impl(int device, bool fp32, int m, int n, const void* A, double tol, int max_cols,
                             int32_t* kckk, void* U, void* V, hipStream_t st);
void apply_compressed(bem_op* op, int nrhs, const zd* x_dev, int64_t x_l_stride, zd* y_dev, hipStream_t st);
void apply_weighted_compressed(bem_op* op, const zd* W_dev, zd* y_dev, hipStream_t st);
// y_l = A(s_l)^T x_l (plain transpose), x, y [nrhs][L][3K] mesh order
void apply_compressed_t(bem_op* op, int nrhs, const zd* x_dev, zd* y_dev, hipStream_t st);
// y = scale sum_l A(s_l) x (the weighted sum with one vector for every frequency)
void apply_sum_compressed(bem_op* op, const zd* x_dev, double scale, zd* y_dev, hipStream_t st);
void compressed_blocks(const bem_op* op, int64_t* n, int64_t* rows, int32_t* perm);
void compressed_freq_hist(const bem_op* op, int64_t* hist);
void destroy_compressed(CompressedOp* c);
// batched products of several compressed operators with one L (compress.cpp)
struct BatchPlan;
BatchPlan* batch_create(bem_op* const* ops, int nops, int nrhs, int flags, hipStream_t st);
void batch_apply(BatchPlan* P, const zd* const* x, zd* const* y, hipStream_t st);
void batch_info(const BatchPlan* P, bem_batch_info* info);
void batch_destroy(BatchPlan* P);
}  // namespace bem
