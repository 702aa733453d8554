// api.cpp -- the extern "C" entry points of libbem: context, mesh/material/frequency
// set-up with validation, the raw entry generator, dense assembly and products, and the
// dispatch to compression (compress.cpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>

#include "host.hpp"
#include "solve.hpp"

using namespace bem;

#pragma clang fp contract(off)

namespace {

const char* kVersion = "libbem 0.1 (gfx950)";

using api_error = bem::ApiError;

int fail(bem_ctx* ctx, int code, const std::string& msg)
{
    if (ctx) ctx->err = msg;
    return code;
}

// Runs f() and converts exceptions into return codes + messages.
template <typename F>
int guarded(bem_ctx* ctx, F&& f)
{
    try {
        if (ctx) ctx->err.clear();
        return f();
    } catch (const api_error& e) {
        return fail(ctx, e.code, e.what());
    } catch (const DevBuf::bem_nomem& e) {
        return fail(ctx, BEM_ERR_NOMEM, e.what());
    } catch (const bem_hip_error& e) {
        return fail(ctx, e.code == hipErrorOutOfMemory ? BEM_ERR_NOMEM : BEM_ERR_HIP, e.what());
    } catch (const std::bad_alloc&) {
        return fail(ctx, BEM_ERR_NOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(ctx, BEM_ERR_ARG, e.what());
    } catch (...) {
        return fail(ctx, BEM_ERR_ARG, "unknown error");
    }
}

void need_device(const bem_ctx* ctx)
{
    if (ctx->device < 0) throw api_error(BEM_ERR_NODEVICE, "host-only context (device = -1)");
    BEM_HIP_TRY(hipSetDevice(ctx->device));
}

// the dense and matrix-free operators couple every pair of elements: not for a context of
// several components (their operators are block diagonal; bem_compress forms them)
void need_one_component(const bem_ctx* ctx)
{
    if (ctx->hgeo.ncomp > 1) throw api_error(BEM_ERR_STATE, "several mesh components: use bem_compress");
}

void need_state(const bem_ctx* ctx, bool freq = true)
{
    if (!ctx->mesh_set) throw api_error(BEM_ERR_STATE, "mesh not set");
    if (!ctx->mat_set) throw api_error(BEM_ERR_STATE, "material not set");
    if (freq && !ctx->freq_set) throw api_error(BEM_ERR_STATE, "frequencies not set");
}

// Gauss-Legendre rule on [-1, 1]: Newton iteration on P_n with the derivative from
// P_n' = n (x P_n - P_{n-1}) / (x^2 - 1); nodes in increasing order.
void gauss_legendre(int n, double* x, double* w)
{
    for (int k = 0; k < n; ++k) {
        // Tricomi-type initial guess for the k-th largest root, mirrored to ascending order
        double z = std::cos(M_PI * (4.0 * k + 3.0) / (4.0 * n + 2.0));
        double pn = 0, pn1 = 0;
        for (int it = 0; it < 64; ++it) {
            double p0 = 1.0, p1 = z;
            if (n == 1) {
                pn = z;
                pn1 = 1.0;
            } else {
                for (int m = 2; m <= n; ++m) {
                    double p2 = ((2 * m - 1) * z * p1 - (m - 1) * p0) / m;
                    p0 = p1;
                    p1 = p2;
                }
                pn = p1;
                pn1 = p0;
            }
            double d = n * (z * pn - pn1) / (z * z - 1.0);
            double step = pn / d;
            z -= step;
            if (std::fabs(step) <= 4e-16 * std::fabs(z) + 1e-300) break;
        }
        double p0 = 1.0, p1 = z;
        if (n == 1) {
            pn = z;
            pn1 = 1.0;
        } else {
            for (int m = 2; m <= n; ++m) {
                double p2 = ((2 * m - 1) * z * p1 - (m - 1) * p0) / m;
                p0 = p1;
                p1 = p2;
            }
            pn = p1;
            pn1 = p0;
        }
        double d = n * (z * pn - pn1) / (z * z - 1.0);
        x[n - 1 - k] = z;
        w[n - 1 - k] = 2.0 / ((1.0 - z * z) * d * d);
    }
}

// 7-point degree-5 triangle rule (barycentric), weights summing to 1.
void tri7(double* b, double* w)
{
    const double r15 = std::sqrt(15.0);
    const double p1 = (6.0 - r15) / 21.0, p2 = (6.0 + r15) / 21.0;
    const double w1 = (155.0 - r15) / 1200.0, w2 = (155.0 + r15) / 1200.0;
    const double pts[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3},
                              {1.0 - 2 * p1, p1, p1}, {p1, 1.0 - 2 * p1, p1}, {p1, p1, 1.0 - 2 * p1},
                              {1.0 - 2 * p2, p2, p2}, {p2, 1.0 - 2 * p2, p2}, {p2, p2, 1.0 - 2 * p2}};
    const double ws[7] = {0.225, w1, w1, w1, w2, w2, w2};
    for (int q = 0; q < 7; ++q) {
        for (int k = 0; k < 3; ++k) b[3 * q + k] = pts[q][k];
        w[q] = ws[q];
    }
}

void rebuild_quadtab(bem_ctx* ctx)
{
    QuadTab& Q = ctx->qtab;
    Q.near_on = ctx->quad.near_on ? 1 : 0;
    Q.r1sq = ctx->quad.near_r1 * ctx->quad.near_r1;
    Q.r2sq = ctx->quad.near_r2 * ctx->quad.near_r2;
    Q.nt = ctx->quad.self_nt;
    Q.nr = ctx->quad.self_nr;
    gauss_legendre(Q.nt, Q.tx, Q.tw);
    gauss_legendre(Q.nr, Q.rx, Q.rw);
    Q.crho = 0.0;
    for (int k = 0; k < Q.nr; ++k) Q.crho += Q.rw[k] / (1.0 + Q.rx[k]);
    tri7(Q.b7, Q.w7);
}

template <typename T>
Mat<T> make_mat(double rho, double c1, double c2)
{
    Mat<T> m;
    m.c1 = (T)c1;
    m.c2 = (T)c2;
    m.ic1 = (T)(1.0 / c1);
    m.ic2 = (T)(1.0 / c2);
    m.ic1s = (T)(1.0 / (c1 * c1));
    m.ic2s = (T)(1.0 / (c2 * c2));
    m.lamc = (T)(c1 * c1 - 2.0 * c2 * c2);
    m.c2s = (T)(c2 * c2);
    m.inv4pirho = (T)(1.0 / (4.0 * M_PI * rho));
    m.inv4pi = (T)(1.0 / (4.0 * M_PI));
    m.gcoef = (T)(c2 * c2 / (4.0 * M_PI * c1 * c1));
    return m;
}

// Host staging of a caller buffer: device pointer as is, host buffers copied.
struct Staged {
    DevBuf buf;
    void* dev = nullptr;
};

void stage_in(Staged& s, const void* src, size_t bytes, bool is_dev, hipStream_t st)
{
    if (is_dev || bytes == 0) {
        s.dev = const_cast<void*>(src);
        return;
    }
    s.buf.alloc(bytes);
    BEM_HIP_TRY(hipMemcpyAsync(s.buf.p, src, bytes, hipMemcpyHostToDevice, st));
    s.dev = s.buf.p;
}

void stage_out(Staged& s, void* dst, size_t bytes, bool is_dev)
{
    if (is_dev || bytes == 0) {
        s.dev = dst;
        return;
    }
    s.buf.alloc(bytes);
    s.dev = s.buf.p;
}

void finish_out(const Staged& s, void* dst, size_t bytes, bool is_dev, hipStream_t st)
{
    if (is_dev || bytes == 0) return;
    BEM_HIP_TRY(hipMemcpyAsync(dst, s.dev, bytes, hipMemcpyDeviceToHost, st));
    BEM_HIP_TRY(hipStreamSynchronize(st));
}

}  // namespace

// ---------------------------------------------------------------- internal helpers

void bem::DevGeo::upload(const HostGeo& h, const int* perm, hipStream_t st)
{
    const int K = h.K;
    // 8 arrays of K, 3 of 3K (vertices), 4 of 7K (rule)
    size_t n = (size_t)K * (8 + 9 + 28);
    std::vector<double> tmp(n);
    auto src = [&](const std::vector<double>& v, int stride_rows, size_t off) {
        for (int r = 0; r < stride_rows; ++r)
            for (int e = 0; e < K; ++e) tmp[off + (size_t)r * K + e] = v[(size_t)r * K + (perm ? perm[e] : e)];
    };
    size_t o = 0;
    const std::vector<double>* one[8] = {&h.cx, &h.cy, &h.cz, &h.nx, &h.ny, &h.nz, &h.area, &h.lmax2};
    size_t offs[15];
    for (int a = 0; a < 8; ++a) {
        offs[a] = o;
        src(*one[a], 1, o);
        o += K;
    }
    const std::vector<double>* three[3] = {&h.vx, &h.vy, &h.vz};
    for (int a = 0; a < 3; ++a) {
        offs[8 + a] = o;
        src(*three[a], 3, o);
        o += 3 * (size_t)K;
    }
    const std::vector<double>* seven[4] = {&h.gx, &h.gy, &h.gz, &h.gw};
    for (int a = 0; a < 4; ++a) {
        offs[11 + a] = o;
        src(*seven[a], 7, o);
        o += 7 * (size_t)K;
    }
    buf.alloc(n * sizeof(double));
    BEM_HIP_TRY(hipMemcpyAsync(buf.p, tmp.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
    BEM_HIP_TRY(hipStreamSynchronize(st));
    const double* d = buf.as<double>();
    geo.K = K;
    geo.cx = d + offs[0];
    geo.cy = d + offs[1];
    geo.cz = d + offs[2];
    geo.nx = d + offs[3];
    geo.ny = d + offs[4];
    geo.nz = d + offs[5];
    geo.area = d + offs[6];
    geo.lmax2 = d + offs[7];
    geo.vx = d + offs[8];
    geo.vy = d + offs[9];
    geo.vz = d + offs[10];
    geo.gx = d + offs[11];
    geo.gy = d + offs[12];
    geo.gz = d + offs[13];
    geo.gw = d + offs[14];
}

bem::DevCtx bem_ctx::devctx(const bem::Geo& g, const int* perm) const
{
    DevCtx c;
    c.geo = g;
    c.md = make_mat<double>(rho, cp, cs);
    c.mf = make_mat<float>(rho, cp, cs);
    c.qt = qtab;
    c.fr = freq;
    c.table = table;
    c.perm = perm;
    return c;
}

bem_op::~bem_op()
{
    if (comp) bem::destroy_compressed(comp);
    comp = nullptr;
    if (ctx) ctx->live_ops--;
}

// ---------------------------------------------------------------- C-ABI

extern "C" {

const char* bem_version(void) { return kVersion; }

int bem_create(bem_ctx** out, int32_t device)
{
    if (!out) return BEM_ERR_ARG;
    *out = nullptr;
    bem_ctx* ctx = nullptr;
    try {
        ctx = new bem_ctx();
    } catch (...) {
        return BEM_ERR_NOMEM;
    }
    ctx->device = device;
    rebuild_quadtab(ctx);
    if (device >= 0) {
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || device >= n) {
            (void)hipGetLastError();
            delete ctx;
            return BEM_ERR_NODEVICE;
        }
        if (hipSetDevice(device) != hipSuccess) {
            delete ctx;
            return BEM_ERR_HIP;
        }
        // device address of the no-allocation scratch, once per device; a failure here is
        // reported by bem_aca_matrix_noalloc, which looks it up again
        try {
            (void)bem::noalloc_scratch(device);
        } catch (...) {
            (void)hipGetLastError();
        }
    }
    *out = ctx;
    return BEM_OK;
}

int bem_destroy(bem_ctx* ctx)
{
    if (!ctx) return BEM_ERR_ARG;
    if (ctx->live_ops > 0) return fail(ctx, BEM_ERR_STATE, "operators of this context are still alive");
    if (ctx->device >= 0) (void)hipSetDevice(ctx->device);
    delete ctx;
    return BEM_OK;
}

const char* bem_last_error(const bem_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int bem_set_stream(bem_ctx* ctx, void* hip_stream)
{
    if (!ctx) return BEM_ERR_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return BEM_OK;
}

int bem_set_mesh(bem_ctx* ctx, const double* nodes, int64_t n_nodes, const int32_t* tris, int64_t K)
{
    if (!ctx) return BEM_ERR_ARG;
    return guarded(ctx, [&]() -> int {
        if (K < 1 || n_nodes < 3 || !nodes || !tris) throw api_error(BEM_ERR_MESH, "need K >= 1 triangles and >= 3 nodes");
        if (K > (int64_t)1 << 28) throw api_error(BEM_ERR_MESH, "too many triangles");
        for (int64_t e = 0; e < 3 * K; ++e)
            if (tris[e] < 0 || tris[e] >= n_nodes)
                throw api_error(BEM_ERR_MESH, "triangle " + std::to_string(e / 3) + " has node index out of range");
        for (int64_t e = 0; e < 3 * n_nodes; ++e)
            if (!std::isfinite(nodes[e])) throw api_error(BEM_ERR_MESH, "non-finite node coordinate");
        HostGeo g;
        g.K = (int)K;
        auto res = [&](std::vector<double>& v, size_t n) { v.assign(n, 0.0); };
        for (auto* v : {&g.cx, &g.cy, &g.cz, &g.nx, &g.ny, &g.nz, &g.area, &g.lmax2}) res(*v, K);
        for (auto* v : {&g.vx, &g.vy, &g.vz}) res(*v, 3 * K);
        for (auto* v : {&g.gx, &g.gy, &g.gz, &g.gw}) res(*v, 7 * K);
        double b7[21], w7[7];
        tri7(b7, w7);
        for (int64_t e = 0; e < K; ++e) {
            double V[3][3];
            for (int a = 0; a < 3; ++a)
                for (int k = 0; k < 3; ++k) V[a][k] = nodes[3 * (int64_t)tris[3 * e + a] + k];
            // centroid: ((v0 + v1) + v2) / 3
            g.cx[e] = (V[0][0] + V[1][0] + V[2][0]) / 3.0;
            g.cy[e] = (V[0][1] + V[1][1] + V[2][1]) / 3.0;
            g.cz[e] = (V[0][2] + V[1][2] + V[2][2]) / 3.0;
            double u[3], w[3];
            for (int k = 0; k < 3; ++k) {
                u[k] = V[1][k] - V[0][k];
                w[k] = V[2][k] - V[0][k];
            }
            double n[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
            double nl = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
            double l2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                int b = (a + 1) % 3;
                double dx = V[b][0] - V[a][0], dy = V[b][1] - V[a][1], dz = V[b][2] - V[a][2];
                double q = dx * dx + dy * dy + dz * dz;
                if (q > l2) l2 = q;
            }
            if (!(nl > 1e-12 * l2)) throw api_error(BEM_ERR_MESH, "triangle " + std::to_string(e) + " is degenerate");
            g.area[e] = 0.5 * nl;
            g.nx[e] = n[0] / nl;
            g.ny[e] = n[1] / nl;
            g.nz[e] = n[2] / nl;
            g.lmax2[e] = l2;
            for (int a = 0; a < 3; ++a) {
                g.vx[(size_t)a * K + e] = V[a][0];
                g.vy[(size_t)a * K + e] = V[a][1];
                g.vz[(size_t)a * K + e] = V[a][2];
            }
            for (int q = 0; q < 7; ++q) {
                const double* b = b7 + 3 * q;
                g.gx[(size_t)q * K + e] = b[0] * V[0][0] + b[1] * V[1][0] + b[2] * V[2][0];
                g.gy[(size_t)q * K + e] = b[0] * V[0][1] + b[1] * V[1][1] + b[2] * V[2][1];
                g.gz[(size_t)q * K + e] = b[0] * V[0][2] + b[1] * V[1][2] + b[2] * V[2][2];
                g.gw[(size_t)q * K + e] = w7[q] * g.area[e];
            }
        }
        ctx->nodes.assign(nodes, nodes + 3 * n_nodes);
        ctx->tris.assign(tris, tris + 3 * K);
        ctx->tris_dev.release();  // re-uploaded on first use
        ctx->hgeo = std::move(g);  // one component until bem_set_components
        if (ctx->device >= 0) {
            need_device(ctx);
            ctx->dgeo.upload(ctx->hgeo, nullptr, ctx->stream);
        }
        ctx->mesh_set = true;
        return BEM_OK;
    });
}

int bem_set_material(bem_ctx* ctx, double rho, double cp, double cs)
{
    if (!ctx) return BEM_ERR_ARG;
    return guarded(ctx, [&]() -> int {
        if (!(std::isfinite(rho) && std::isfinite(cp) && std::isfinite(cs)) || !(rho > 0) || !(cs > 0) || !(cp > cs))
            throw api_error(BEM_ERR_MATERIAL, "need rho > 0 and cp > cs > 0");
        ctx->rho = rho;
        ctx->cp = cp;
        ctx->cs = cs;
        ctx->mat_set = true;
        if (cp * cp < 4.0 / 3.0 * cs * cs) {
            ctx->err = "cp^2 < 4/3 cs^2: negative bulk modulus";
            return BEM_WARN_BULK;
        }
        return BEM_OK;
    });
}

int bem_set_frequencies(bem_ctx* ctx, const double* s, int32_t L)
{
    if (!ctx) return BEM_ERR_ARG;
    return guarded(ctx, [&]() -> int {
        if (L < 1 || !s) throw api_error(BEM_ERR_FREQ, "need L >= 1 frequencies");
        std::vector<zd> v(L);
        for (int l = 0; l < L; ++l) {
            v[l] = {s[2 * l], s[2 * l + 1]};
            if (!std::isfinite(v[l].re) || !std::isfinite(v[l].im) || !(v[l].re > 0))
                throw api_error(BEM_ERR_FREQ, "frequency " + std::to_string(l) + " must have a finite, positive real part");
        }
        ctx->s = v;
        if (ctx->device >= 0) {
            need_device(ctx);
            size_t bytes = (size_t)L * (2 * sizeof(zd) + 2 * sizeof(zf));
            std::vector<char> tmp(bytes);
            zd* sd = (zd*)tmp.data();
            zd* sid = sd + L;
            zf* sf = (zf*)(sid + L);
            zf* sif = sf + L;
            for (int l = 0; l < L; ++l) {
                sd[l] = v[l];
                sid[l] = zdiv(zd{1.0, 0.0}, v[l]);
                sf[l] = {(float)v[l].re, (float)v[l].im};
                sif[l] = {(float)sid[l].re, (float)sid[l].im};
            }
            ctx->fbuf.alloc(bytes);
            BEM_HIP_TRY(hipMemcpyAsync(ctx->fbuf.p, tmp.data(), bytes, hipMemcpyHostToDevice, ctx->stream));
            BEM_HIP_TRY(hipStreamSynchronize(ctx->stream));
            zd* d = ctx->fbuf.as<zd>();
            ctx->freq.s = d;
            ctx->freq.sinv = d + L;
            ctx->freq.sf = (const zf*)(d + 2 * L);
            ctx->freq.sinvf = (const zf*)(d + 2 * L) + L;
        }
        ctx->freq.L = L;
        ctx->freq_set = true;
        return BEM_OK;
    });
}

int bem_freq_pairs(const bem_ctx* ctx, int32_t* n_pairs)
{
    if (!ctx || !n_pairs) return BEM_ERR_ARG;
    int n = 0, L = (int)ctx->s.size();
    for (int a = 0; a < L; ++a)
        for (int b = 0; b < L; ++b)
            if (a != b && ctx->s[a].re == ctx->s[b].re && ctx->s[a].im == -ctx->s[b].im && ctx->s[a].im != 0.0) {
                ++n;
                break;
            }
    *n_pairs = n;
    return BEM_OK;
}

int bem_set_quadrature(bem_ctx* ctx, const bem_quad* q)
{
    if (!ctx) return BEM_ERR_ARG;
    bem_quad d{0, 1.5, 3.0, 8, 8};
    if (q) {
        if (q->self_nt < 1 || q->self_nt > 16 || q->self_nr < 1 || q->self_nr > 16 || !(q->near_r1 >= 0) ||
            !(q->near_r2 >= q->near_r1))
            return fail(ctx, BEM_ERR_ARG, "self_nt/self_nr must be in 1..16 and 0 <= near_r1 <= near_r2");
        d = *q;
    }
    ctx->quad = d;
    rebuild_quadtab(ctx);
    return BEM_OK;
}

int bem_set_entry_table(bem_ctx* ctx, const void* table_dev)
{
    if (!ctx) return BEM_ERR_ARG;
    ctx->table = (const zd*)table_dev;
    return BEM_OK;
}

int bem_set_components(bem_ctx* ctx, const int32_t* comp, int32_t ncomp)
{
    if (!ctx) return BEM_ERR_ARG;
    return guarded(ctx, [&]() -> int {
        if (!ctx->mesh_set) throw api_error(BEM_ERR_STATE, "mesh not set");
        HostGeo& g = ctx->hgeo;
        if (!comp || ncomp <= 1) {
            g.comp.clear();
            g.ncomp = 1;
            return BEM_OK;
        }
        std::vector<int> c(comp, comp + g.K), seen(ncomp, 0);
        for (int e = 0; e < g.K; ++e) {
            if (c[e] < 0 || c[e] >= ncomp) throw api_error(BEM_ERR_ARG, "component index out of range");
            seen[c[e]] = 1;
        }
        for (int q = 0; q < ncomp; ++q)
            if (!seen[q]) throw api_error(BEM_ERR_ARG, "component " + std::to_string(q) + " has no element");
        g.comp = std::move(c);
        g.ncomp = ncomp;
        return BEM_OK;
    });
}

int bem_entries(bem_ctx* ctx, int32_t op, int32_t prec, int64_t n, const int32_t* i, const int32_t* j,
                const int32_t* l, void* out, int32_t flags)
{
    if (!ctx) return BEM_ERR_ARG;
    return guarded(ctx, [&]() -> int {
        if (op < 0 || op > BEM_OP_KL2 || (prec != BEM_PREC_F64 && prec != BEM_PREC_MIXED) || n < 0)
            throw api_error(BEM_ERR_ARG, "bad op, prec or n");
        if (op >= BEM_OP_KL0 && prec != BEM_PREC_F64) throw api_error(BEM_ERR_ARG, "linear-basis entries are FP64");
        need_state(ctx);
        need_device(ctx);
        if (op == BEM_OP_TABLE && !ctx->table) throw api_error(BEM_ERR_STATE, "no entry table set");
        if (n == 0) return BEM_OK;
        if (!i || !j || !l || !out) throw api_error(BEM_ERR_ARG, "null buffer");
        bool dev = (flags & BEM_DEVICE_PTR) != 0;
        if (!dev) {
            for (int64_t e = 0; e < n; ++e)
                if (i[e] < 0 || i[e] >= ctx->hgeo.K || j[e] < 0 || j[e] >= ctx->hgeo.K || l[e] < 0 ||
                    l[e] >= ctx->freq.L)
                    throw api_error(BEM_ERR_ARG, "index out of range at entry " + std::to_string(e));
        }
        hipStream_t st = ctx->stream;
        Staged si, sj, sl, so;
        size_t ib = (size_t)n * sizeof(int32_t), ob = (size_t)n * 9 * sizeof(zd);
        stage_in(si, i, ib, dev, st);
        stage_in(sj, j, ib, dev, st);
        stage_in(sl, l, ib, dev, st);
        stage_out(so, out, ob, dev);
        DevCtx c = ctx->devctx(ctx->dgeo.geo, nullptr);
        launch_entries(c, op, prec == BEM_PREC_MIXED, n, (const int32_t*)si.dev, (const int32_t*)sj.dev,
                       (const int32_t*)sl.dev, (zd*)so.dev, st);
        finish_out(so, out, ob, dev, st);
        return BEM_OK;
    });
}

int bem_assemble_dense(bem_ctx* ctx, int32_t op, int32_t prec, bem_op** out)
{
    if (!ctx || !out) return BEM_ERR_ARG;
    *out = nullptr;
    return guarded(ctx, [&]() -> int {
        if (op < 0 || op > 3 || (prec != BEM_PREC_F64 && prec != BEM_PREC_MIXED))
            throw api_error(BEM_ERR_ARG, "bad op or prec");
        need_state(ctx);
        need_device(ctx);
        need_one_component(ctx);
        if (op == BEM_OP_TABLE && !ctx->table) throw api_error(BEM_ERR_STATE, "no entry table set");
        int K = ctx->hgeo.K, L = ctx->freq.L;
        if (K > 65535) throw api_error(BEM_ERR_ARG, "dense assembly is limited to K <= 65535");
        auto t0 = std::chrono::steady_clock::now();
        std::unique_ptr<bem_op> o(new bem_op());
        o->ctx = ctx;
        ctx->live_ops++;
        o->op = op;
        o->prec = prec;
        o->kind = 0;
        o->K = K;
        o->L = L;
        size_t M = 3 * (size_t)K;
        o->dense.alloc((size_t)L * M * M * sizeof(zd));
        DevCtx c = ctx->devctx(ctx->dgeo.geo, nullptr);
        launch_dense_assemble(c, op, prec == BEM_PREC_MIXED, o->dense.as<zd>(), ctx->stream);
        BEM_HIP_TRY(hipStreamSynchronize(ctx->stream));
        bem_stats& st = o->stats;
        st.n_blocks = 1;
        st.n_near = 1;
        st.rank_min = st.rank_max = L;
        st.rank_mean = L;
        st.bytes = (int64_t)o->dense.bytes;
        st.compression_rate = 1.0;
        st.entries_generated = (int64_t)K * K * L;
        st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *out = o.release();
        return BEM_OK;
    });
}

int bem_matrix_free(bem_ctx* ctx, int32_t op, bem_op** out)
{
    if (!ctx || !out) return BEM_ERR_ARG;
    *out = nullptr;
    return guarded(ctx, [&]() -> int {
        if (op != BEM_OP_V && op != BEM_OP_K && op != BEM_OP_HK) throw api_error(BEM_ERR_ARG, "op must be V, K or HK");
        need_state(ctx);
        need_device(ctx);
        need_one_component(ctx);
        std::unique_ptr<bem_op> o(new bem_op());
        o->ctx = ctx;
        ctx->live_ops++;
        o->op = op;
        o->prec = BEM_PREC_F64;
        o->kind = 2;
        o->K = ctx->hgeo.K;
        o->L = ctx->freq.L;
        o->stats.n_blocks = 1;
        o->stats.n_near = 1;
        *out = o.release();
        return BEM_OK;
    });
}

int bem_op_dense_copy(const bem_op* op, void* dst, int32_t flags)
{
    if (!op || !dst) return BEM_ERR_ARG;
    bem_ctx* ctx = op->ctx;
    return guarded(ctx, [&]() -> int {
        if (op->kind != 0) throw api_error(BEM_ERR_ARG, "operator is not dense");
        need_device(ctx);
        hipMemcpyKind k = (flags & BEM_DEVICE_PTR) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        BEM_HIP_TRY(hipMemcpyAsync(dst, op->dense.p, op->dense.bytes, k, ctx->stream));
        if (!(flags & BEM_DEVICE_PTR)) BEM_HIP_TRY(hipStreamSynchronize(ctx->stream));
        return BEM_OK;
    });
}

int bem_compress(bem_ctx* ctx, int32_t op, const bem_aca_opts* opts, bem_op** out)
{
    if (!ctx || !out) return BEM_ERR_ARG;
    *out = nullptr;
    return guarded(ctx, [&]() -> int {
        if (op < 0 || op > 3) throw api_error(BEM_ERR_ARG, "bad op");
        need_state(ctx);
        need_device(ctx);
        if (op == BEM_OP_TABLE && !ctx->table) throw api_error(BEM_ERR_STATE, "no entry table set");
        bem_aca_opts o{1e-6, 0.0, 1.5, 64, BEM_PREC_F64, 1e-5, 0, 48, 0, BEM_FACES_AFTER};
        if (opts) o = *opts;
        if (!(o.eps3d > 0 && o.eps3d < 1) || !(o.eta > 0) || o.leaf < 1 ||
            (o.prec != BEM_PREC_F64 && o.prec != BEM_PREC_MIXED) || o.pool_bytes < 0 || o.far_dense_max < 0 ||
            o.aca_rounds < 0 || o.aca_rounds > 64 || (o.face_order != BEM_FACES_AFTER && o.face_order != BEM_FACES_IN_LOOP))
            throw api_error(BEM_ERR_ARG, "bad compression options");
        if (!(o.eps_aca > 0)) o.eps_aca = o.eps3d / 100.0;
        if (!(o.mixed_eps_floor > 0)) o.mixed_eps_floor = 1e-5;
        std::unique_ptr<bem_op> res(new bem_op());
        res->ctx = ctx;
        ctx->live_ops++;
        res->op = op;
        res->prec = o.prec;
        res->kind = 1;
        res->K = ctx->hgeo.K;
        res->L = ctx->freq.L;
        int rc = compress_impl(ctx, op, o, res.get());
        if (rc < 0) return rc;
        *out = res.release();
        return rc;
    });
}

int bem_aca_matrix(bem_ctx* ctx, int32_t prec, int32_t m, int32_t n, const void* A, double tol, int32_t max_cols,
                   int32_t* kc, int32_t* kk, void* U, void* V)
{
    if (!ctx) return BEM_ERR_ARG;
    return guarded(ctx, [&]() -> int {
        if (m < 1 || n < 1 || (int64_t)m * n > (1 << 22) || (prec != BEM_PREC_F64 && prec != BEM_PREC_MIXED) ||
            !(tol >= 0) || !A)
            throw api_error(BEM_ERR_ARG, "bad bem_aca_matrix arguments");
        need_device(ctx);
        int c = 0, k = 0;
        aca_matrix_impl(ctx, prec == BEM_PREC_MIXED, m, n, A, tol, max_cols, &c, &k, U, V);
        if (kc) *kc = c;
        if (kk) *kk = k;
        return BEM_OK;
    });
}

int bem_aca_matrix_noalloc(bem_ctx* ctx, int32_t prec, int32_t m, int32_t n, const void* A, double tol,
                           int32_t max_cols, int32_t* kc_kk, void* U, void* V)
{
    if (!ctx) return BEM_ERR_ARG;
    return guarded(ctx, [&]() -> int {
        if (m < 1 || n < 1 || m > BEM_ACA_NOALLOC_MAX_ELEMENTS || n > BEM_ACA_NOALLOC_MAX_ELEMENTS ||
            (prec != BEM_PREC_F64 && prec != BEM_PREC_MIXED) || !(tol >= 0) || !A || !kc_kk || !U || !V)
            throw api_error(BEM_ERR_ARG, "bad bem_aca_matrix_noalloc arguments");
        need_device(ctx);
        aca_matrix_noalloc_impl(ctx->device, prec == BEM_PREC_MIXED, m, n, A, tol, max_cols, kc_kk, U, V,
                                ctx->stream);
        return BEM_OK;
    });
}

int bem_op_stats(const bem_op* op, bem_stats* st)
{
    if (!op || !st) return BEM_ERR_ARG;
    *st = op->stats;
    return BEM_OK;
}

int bem_apply(bem_op* op, int32_t nrhs, const void* x, void* y, int32_t flags)
{
    if (!op) return BEM_ERR_ARG;
    bem_ctx* ctx = op->ctx;
    return guarded(ctx, [&]() -> int {
        if (nrhs < 1 || !x || !y) throw api_error(BEM_ERR_ARG, "need nrhs >= 1 and buffers");
        need_device(ctx);
        bool dev = (flags & BEM_DEVICE_PTR) != 0;
        bool shared = (flags & BEM_SHARED_X) != 0;
        const bool trans = (flags & BEM_TRANSPOSE) != 0;
        if (trans && shared) throw api_error(BEM_ERR_ARG, "BEM_TRANSPOSE with BEM_SHARED_X");
        if (op->kind == 2) {
            if (shared) throw api_error(BEM_ERR_ARG, "BEM_SHARED_X with a matrix-free operator");
            need_state(ctx);
            need_one_component(ctx);
            if (ctx->hgeo.K != op->K || ctx->freq.L != op->L)
                throw api_error(BEM_ERR_STATE, "the context's mesh or contour changed size since bem_matrix_free");
        }
        size_t M = 3 * (size_t)op->K;
        size_t xb = (size_t)nrhs * (shared ? 1 : op->L) * M * sizeof(zd);
        size_t yb = (size_t)nrhs * op->L * M * sizeof(zd);
        hipStream_t st = ctx->stream;
        Staged sx, sy;
        stage_in(sx, x, xb, dev, st);
        stage_out(sy, y, yb, dev);
        int64_t xls = shared ? 0 : (int64_t)M;
        if (op->kind == 2) {
            launch_mf_apply(ctx->devctx(ctx->dgeo.geo, nullptr), op->op, trans, nrhs, (const zd*)sx.dev, (zd*)sy.dev,
                            st);
        } else if (trans && op->kind == 0)
            launch_dense_apply_t(op->dense.as<zd>(), (int)M, op->L, nrhs, (const zd*)sx.dev, (zd*)sy.dev, st);
        else if (trans)
            apply_compressed_t(op, nrhs, (const zd*)sx.dev, (zd*)sy.dev, st);
        else if (op->kind == 0)
            launch_dense_apply(op->dense.as<zd>(), (int)M, op->L, nrhs, (const zd*)sx.dev, xls, (zd*)sy.dev, st);
        else
            apply_compressed(op, nrhs, (const zd*)sx.dev, xls, (zd*)sy.dev, st);
        finish_out(sy, y, yb, dev, st);
        return BEM_OK;
    });
}

namespace {

// y = A x for [nrhs][L][3K] device buffers (mesh order)
void op_apply(bem_op* op, int nrhs, const zd* x, zd* y, hipStream_t st, bool trans = false)
{
    const size_t M = 3 * (size_t)op->K;
    if (op->kind == 2) {
        const bem_ctx* c = op->ctx;
        if (c->hgeo.K != op->K || c->freq.L != op->L || c->hgeo.ncomp > 1)
            throw api_error(BEM_ERR_STATE, "the context of a matrix-free operator changed its mesh or contour size");
        launch_mf_apply(c->devctx(c->dgeo.geo, nullptr), op->op, trans, nrhs, x, y, st);
    } else if (trans && op->kind == 0)
        launch_dense_apply_t(op->dense.as<zd>(), (int)M, op->L, nrhs, x, y, st);
    else if (trans)
        apply_compressed_t(op, nrhs, x, y, st);
    else if (op->kind == 0)
        launch_dense_apply(op->dense.as<zd>(), (int)M, op->L, nrhs, x, (int64_t)M, y, st);
    else
        apply_compressed(op, nrhs, x, (int64_t)M, y, st);
}

}  // namespace

int bem_solve(bem_op* A, bem_op* A_inner, int32_t nrhs, const void* b, void* x, int32_t flags,
              const bem_solve_opts* opts, bem_solve_stats* stats)
{
    if (!A) return BEM_ERR_ARG;
    bem_ctx* ctx = A->ctx;
    return guarded(ctx, [&]() -> int {
        const auto t0 = std::chrono::steady_clock::now();
        if (nrhs < 1 || !b || !x) throw api_error(BEM_ERR_ARG, "need nrhs >= 1 and buffers");
        if (A_inner && (A_inner->ctx->device != ctx->device || A_inner->K != A->K || A_inner->L != A->L))
            throw api_error(BEM_ERR_ARG, "inner operator of another device or size");
        for (const bem_op* o : {A, A_inner})
            if (o && o->kind == 2 &&
                (o->ctx->hgeo.K != o->K || o->ctx->freq.L != o->L || o->ctx->hgeo.ncomp > 1))
                throw api_error(BEM_ERR_STATE, "the context of a matrix-free operator changed its mesh or contour size");
        bem::SolveParams p;
        if (opts) {
            if (!(opts->tol > 0.0) || !(opts->inner_tol > 0.0 && opts->inner_tol < 1.0) || opts->restart < 1 ||
                opts->max_iter < 1 || opts->max_refine < 0)
                throw api_error(BEM_ERR_ARG, "solve options out of range");
            p.tol = opts->tol;
            p.inner_tol = opts->inner_tol;
            p.restart = opts->restart;
            p.max_iter = opts->max_iter;
            p.max_refine = opts->max_refine;
        }
        need_device(ctx);
        const bool dev = (flags & BEM_DEVICE_PTR) != 0;
        const size_t M = 3 * (size_t)A->K;
        const size_t bytes = (size_t)nrhs * A->L * M * sizeof(zd);
        hipStream_t st = ctx->stream;
        Staged sb, sx;
        stage_in(sb, b, bytes, dev, st);
        stage_out(sx, x, bytes, dev);
        const bool trans = (flags & BEM_TRANSPOSE) != 0;
        bem::DevApply fa = [&](const zd* in, zd* out) { op_apply(A, nrhs, in, out, st, trans); };
        bem::DevApply fi = [&](const zd* in, zd* out) { op_apply(A_inner, nrhs, in, out, st, trans); };
        const bool two = A_inner && A_inner != A;
        const bem::SolveResult R = bem::gmres_refine(fa, two ? fi : fa, (int)M, nrhs * A->L, (const zd*)sb.dev,
                                                     (zd*)sx.dev, p, st);
        finish_out(sx, x, bytes, dev, st);
        if (stats) {
            stats->iterations = R.iterations;
            stats->refinements = R.refinements;
            stats->converged = R.converged ? 1 : 0;
            stats->pad = 0;
            stats->rel_residual = R.rel_residual;
            stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        return R.converged ? BEM_OK : BEM_WARN_NOCONV;
    });
}

int bem_apply_weighted(bem_op* op, const void* W, void* y, int32_t flags)
{
    if (!op) return BEM_ERR_ARG;
    bem_ctx* ctx = op->ctx;
    return guarded(ctx, [&]() -> int {
        if (!W || !y) throw api_error(BEM_ERR_ARG, "null buffer");
        if (op->kind == 2) throw api_error(BEM_ERR_ARG, "weighted sum of a matrix-free operator");
        need_device(ctx);
        bool dev = (flags & BEM_DEVICE_PTR) != 0;
        size_t M = 3 * (size_t)op->K;
        size_t wb = (size_t)op->L * M * sizeof(zd), yb = M * sizeof(zd);
        hipStream_t st = ctx->stream;
        Staged sw, sy;
        stage_in(sw, W, wb, dev, st);
        stage_out(sy, y, yb, dev);
        if (op->kind == 0)
            launch_dense_weighted(op->dense.as<zd>(), (int)M, op->L, (const zd*)sw.dev, (zd*)sy.dev, st);
        else
            apply_weighted_compressed(op, (const zd*)sw.dev, (zd*)sy.dev, st);
        finish_out(sy, y, yb, dev, st);
        return BEM_OK;
    });
}

int bem_op_blocks(const bem_op* op, int64_t* n_blocks, int64_t* rows, int32_t* perm)
{
    if (!op || !n_blocks) return BEM_ERR_ARG;
    if (op->kind != 1) {
        *n_blocks = 1;
        if (rows) {
            int64_t r[8] = {0, op->K, 0, op->K, 0, op->L, 0, 0};
            std::memcpy(rows, r, sizeof(r));
        }
        if (perm)
            for (int e = 0; e < op->K; ++e) perm[e] = e;
        return BEM_OK;
    }
    compressed_blocks(op, n_blocks, rows, perm);
    return BEM_OK;
}

int bem_partition(bem_ctx* ctx, double eta, int32_t leaf, int64_t* n_blocks, int64_t* rows, int32_t* perm)
{
    if (!ctx || !n_blocks) return BEM_ERR_ARG;
    return guarded(ctx, [&]() -> int {
        if (!ctx->mesh_set) throw api_error(BEM_ERR_STATE, "mesh not set");
        if (!(eta > 0) || leaf < 1) throw api_error(BEM_ERR_ARG, "need eta > 0 and leaf >= 1");
        Partition p;
        build_partition(ctx->hgeo, eta, leaf, p);
        *n_blocks = (int64_t)p.blocks.size();
        if (rows)
            for (size_t b = 0; b < p.blocks.size(); ++b) {
                const BlockDesc& d = p.blocks[b];
                int64_t r[8] = {d.rb, d.rs, d.cb, d.cs, d.far, 0, 0, 0};
                std::memcpy(rows + 8 * b, r, sizeof(r));
            }
        if (perm)
            for (int e = 0; e < ctx->hgeo.K; ++e) perm[e] = p.perm[e];
        return BEM_OK;
    });
}

int bem_op_freq_hist(const bem_op* op, int64_t* hist)
{
    if (!op || !hist) return BEM_ERR_ARG;
    if (op->kind != 1) {
        for (int l = 0; l < op->L; ++l) hist[l] = 1;
        return BEM_OK;
    }
    compressed_freq_hist(op, hist);
    return BEM_OK;
}

namespace {

// y = sum_l A(s_l) W[l] on device buffers (W: [L][3K], y: [3K])
void op_apply_weighted(bem_op* op, const zd* W, zd* y, hipStream_t st)
{
    if (op->kind == 0) launch_dense_weighted(op->dense.as<zd>(), 3 * op->K, op->L, W, y, st);
    else apply_weighted_compressed(op, W, y, st);
}

}  // namespace

int bem_cq_dirichlet(bem_op* V, bem_op* H, int32_t N, double dt, double R, const void* g, void* t, int32_t flags,
                     const bem_solve_opts* opts, bem_solve_stats* stats)
{
    if (!V) return BEM_ERR_ARG;
    bem_ctx* ctx = V->ctx;
    return guarded(ctx, [&]() -> int {
        const auto t0 = std::chrono::steady_clock::now();
        const int L = V->L, K = V->K;
        if (!g || !t || N < 1 || N > L) throw api_error(BEM_ERR_ARG, "need buffers and 1 <= N <= L");
        if (H && (H->ctx != ctx || H->K != K || H->L != L)) throw api_error(BEM_ERR_ARG, "H of another context or size");
        if (V->kind == 2 || (H && H->kind == 2)) throw api_error(BEM_ERR_ARG, "time stepping with a matrix-free operator");
        if (!(dt > 0.0) || !(R > 0.0 && R < 1.0)) throw api_error(BEM_ERR_ARG, "need dt > 0 and 0 < R < 1");
        if (flags & ~BEM_DEVICE_PTR) throw api_error(BEM_ERR_ARG, "unknown flags for bem_cq_dirichlet");
        // the contour points must be the BDF2 ones: s_l = delta(z_l) / dt, z_l = R exp(2 pi i l / L)
        std::vector<zd> zinv(L);
        for (int l = 0; l < L; ++l) {
            const std::complex<double> z = std::polar(R, 2.0 * M_PI * l / L);
            const std::complex<double> sl = (1.5 - 2.0 * z + 0.5 * z * z) / dt, sc(ctx->s[l].re, ctx->s[l].im);
            if (std::abs(sl - sc) > 1e-9 * std::abs(sl))
                throw api_error(BEM_ERR_FREQ, "contour point " + std::to_string(l) + " is not delta(z_l)/dt of BDF2");
            const std::complex<double> zi = 1.0 / z;
            zinv[l] = {zi.real(), zi.imag()};
        }
        bem::SolveParams p;
        if (opts) {
            if (!(opts->tol > 0.0) || opts->restart < 1 || opts->max_iter < 1)
                throw api_error(BEM_ERR_ARG, "solve options out of range");
            p.tol = opts->tol;
            p.restart = opts->restart;
            p.max_iter = opts->max_iter;
            p.max_refine = opts->max_refine;
        }
        p.inner_tol = 0.0;  // the inner operator is the fine one
        need_device(ctx);
        const bool dev = (flags & BEM_DEVICE_PTR) != 0;
        const size_t M = 3 * (size_t)K;
        const size_t bytes = (size_t)N * M * sizeof(zd);
        hipStream_t st = ctx->stream;
        Staged sg, stt;
        stage_in(sg, g, bytes, dev, st);
        stage_out(stt, t, bytes, dev);
        DevBuf wt, wg, tmp, tmp2, vb, zb;
        wt.alloc((size_t)L * M * sizeof(zd));
        wg.alloc((size_t)L * M * sizeof(zd));
        tmp.alloc((size_t)L * M * sizeof(zd));
        tmp2.alloc((size_t)L * M * sizeof(zd));
        vb.alloc(3 * M * sizeof(zd));
        zb.alloc((size_t)L * sizeof(zd));
        BEM_HIP_TRY(hipMemsetAsync(wt.p, 0, (size_t)L * M * sizeof(zd), st));
        BEM_HIP_TRY(hipMemsetAsync(wg.p, 0, (size_t)L * M * sizeof(zd), st));
        BEM_HIP_TRY(hipMemcpyAsync(zb.p, zinv.data(), (size_t)L * sizeof(zd), hipMemcpyHostToDevice, st));
        zd* b = vb.as<zd>();
        zd* h = b + M;
        zd* rhs = h + M;
        const zd* gd = (const zd*)sg.dev;
        zd* td = (zd*)stt.dev;
        const double invL = 1.0 / L;
        // omega_0(V) x = sum_l V(s_l) x / L
        bem::DevApply A0 = [&](const zd* in, zd* out) {
            if (V->kind == 1) {
                apply_sum_compressed(V, in, invL, out, st);
            } else {
                launch_cq_fill(tmp2.as<zd>(), nullptr, in, invL, L, (int)M, st);
                op_apply_weighted(V, tmp2.as<zd>(), out, st);
            }
        };
        bem_solve_stats S{};
        S.converged = 1;
        for (int n = 0; n < N; ++n) {
            const zd* gn = gd + (size_t)n * M;
            zd* tn = td + (size_t)n * M;
            // b_n = sum_{j <= n} omega_{n-j}(H) g_j = sum_l H(s_l) (Wg[l] + g_n / L)
            if (H) {
                launch_cq_fill(tmp.as<zd>(), wg.as<zd>(), gn, invL, L, (int)M, st);
                op_apply_weighted(H, tmp.as<zd>(), b, st);
            } else {
                BEM_HIP_TRY(hipMemcpyAsync(b, gn, M * sizeof(zd), hipMemcpyDeviceToDevice, st));
            }
            // history sum_{j < n} omega_{n-j}(V) t_j = sum_l V(s_l) Wt[l] (eq. (3DacaMult))
            op_apply_weighted(V, wt.as<zd>(), h, st);
            launch_axpby(rhs, 1.0, b, -1.0, h, M, st);
            const bem::SolveResult r = bem::gmres_refine(A0, A0, (int)M, 1, rhs, tn, p, st);
            S.iterations += r.iterations;
            S.refinements += r.refinements;
            S.rel_residual = std::max(S.rel_residual, r.rel_residual);
            if (!r.converged) S.converged = 0;
            launch_cq_update(wt.as<zd>(), tn, zb.as<zd>(), invL, L, (int)M, st);
            if (H) launch_cq_update(wg.as<zd>(), gn, zb.as<zd>(), invL, L, (int)M, st);
        }
        finish_out(stt, t, bytes, dev, st);
        BEM_HIP_TRY(hipStreamSynchronize(st));
        S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (stats) *stats = S;
        return S.converged ? BEM_OK : BEM_WARN_NOCONV;
    });
}

int bem_apply_mf(bem_ctx* ctx, int32_t op, int32_t transpose, int32_t nrhs, const void* x, void* y, int32_t flags)
{
    if (!ctx) return BEM_ERR_ARG;
    return guarded(ctx, [&]() -> int {
        need_state(ctx);
        if (op != BEM_OP_V && op != BEM_OP_K && op != BEM_OP_HK) throw api_error(BEM_ERR_ARG, "op must be V, K or HK");
        if (nrhs < 1 || !x || !y) throw api_error(BEM_ERR_ARG, "need nrhs >= 1 and buffers");
        if (flags & ~BEM_DEVICE_PTR) throw api_error(BEM_ERR_ARG, "unknown flags for bem_apply_mf");
        need_device(ctx);
        need_one_component(ctx);
        const bool dev = (flags & BEM_DEVICE_PTR) != 0;
        const size_t bytes = (size_t)nrhs * ctx->freq.L * 3 * (size_t)ctx->hgeo.K * sizeof(zd);
        hipStream_t st = ctx->stream;
        Staged sx, sy;
        stage_in(sx, x, bytes, dev, st);
        stage_out(sy, y, bytes, dev);
        launch_mf_apply(ctx->devctx(ctx->dgeo.geo, nullptr), op, transpose != 0, nrhs, (const zd*)sx.dev, (zd*)sy.dev,
                        st);
        finish_out(sy, y, bytes, dev, st);
        return BEM_OK;
    });
}

int bem_apply_linear_dl(bem_ctx* ctx, int32_t nrhs, const void* g, void* y, int32_t flags)
{
    if (!ctx) return BEM_ERR_ARG;
    return guarded(ctx, [&]() -> int {
        need_state(ctx);
        if (nrhs < 1 || !g || !y) throw api_error(BEM_ERR_ARG, "need nrhs >= 1 and buffers");
        if (flags & ~(BEM_DEVICE_PTR | BEM_FREE_TERM)) throw api_error(BEM_ERR_ARG, "unknown flags for bem_apply_linear_dl");
        need_device(ctx);
        need_one_component(ctx);
        const bool dev = (flags & BEM_DEVICE_PTR) != 0;
        const int K = ctx->hgeo.K;
        const int64_t nn = (int64_t)ctx->nodes.size() / 3;
        const size_t gb = (size_t)nrhs * ctx->freq.L * 3 * (size_t)nn * sizeof(zd);
        const size_t yb = (size_t)nrhs * ctx->freq.L * 3 * (size_t)K * sizeof(zd);
        hipStream_t st = ctx->stream;
        if (!ctx->tris_dev.p) {
            ctx->tris_dev.alloc(sizeof(int32_t) * 3 * (size_t)K);
            BEM_HIP_TRY(hipMemcpyAsync(ctx->tris_dev.p, ctx->tris.data(), sizeof(int32_t) * 3 * (size_t)K,
                                       hipMemcpyHostToDevice, st));
        }
        Staged sg, sy;
        stage_in(sg, g, gb, dev, st);
        stage_out(sy, y, yb, dev);
        launch_mf_apply_kl(ctx->devctx(ctx->dgeo.geo, nullptr), ctx->tris_dev.as<int>(), (int)nn, nrhs,
                           (const zd*)sg.dev, (zd*)sy.dev, (flags & BEM_FREE_TERM) != 0, st);
        finish_out(sy, y, yb, dev, st);
        return BEM_OK;
    });
}

namespace {

// Element results of an adjoint launch to the caller's outputs: per element the 9 vertex
// derivatives of its pairs as column element plus its self terms, the 3 centroid derivatives
// as row element spread over its vertices (fixed order: elements ascending); the material and
// the value from the tiles and the self terms.  drho_scale: d S / d rho = drho_scale * S.
void adjoint_finish(bem_ctx* ctx, const double* sums, const double* tiles, int ntiles, const double* self_out,
                    double drho_scale, double* value, double* grad_nodes, double* grad_mat)
{
    const int K = ctx->hgeo.K;
    hipStream_t st = ctx->stream;
    std::vector<double> hs(12 * (size_t)K), ht(4 * (size_t)ntiles), hself(13 * (size_t)K);
    BEM_HIP_TRY(hipMemcpyAsync(hs.data(), sums, hs.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    BEM_HIP_TRY(hipMemcpyAsync(ht.data(), tiles, ht.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    BEM_HIP_TRY(hipMemcpyAsync(hself.data(), self_out, hself.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    BEM_HIP_TRY(hipStreamSynchronize(st));
    const int64_t nn = (int64_t)ctx->nodes.size() / 3;
    std::vector<double> gn(3 * (size_t)nn, 0.0);
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    for (int t = 0; t < ntiles; ++t)
        for (int k = 0; k < 4; ++k) m[k] += ht[4 * (size_t)t + k];
    for (int e = 0; e < K; ++e) {
        const int32_t* tri = &ctx->tris[3 * (size_t)e];
        const double* gJ = &hs[9 * (size_t)e];
        const double* gI = &hs[9 * (size_t)K + 3 * (size_t)e];
        const double* so = &hself[13 * (size_t)e];
        for (int a = 0; a < 3; ++a)
            for (int k = 0; k < 3; ++k) gn[3 * (size_t)tri[a] + k] += gJ[3 * a + k] + so[3 * a + k] + gI[k] / 3.0;
        m[0] += so[9];
        m[1] += so[10];
        m[2] += so[11];
        m[3] += so[12];
    }
    if (value) {
        value[0] = m[2];
        value[1] = m[3];
    }
    if (grad_nodes) std::copy(gn.begin(), gn.end(), grad_nodes);
    if (grad_mat) {
        grad_mat[0] = drho_scale * m[2];
        grad_mat[1] = m[0];
        grad_mat[2] = m[1];
    }
}

}  // namespace

int bem_adjoint_v(bem_ctx* ctx, int32_t nrhs, const void* w, const void* x, int32_t flags, double* value,
                  double* grad_nodes, double* grad_mat)
{
    if (!ctx) return BEM_ERR_ARG;
    return guarded(ctx, [&]() -> int {
        need_state(ctx);
        if (nrhs < 1 || !w || !x) throw api_error(BEM_ERR_ARG, "need nrhs >= 1 and buffers");
        if (flags & ~BEM_DEVICE_PTR) throw api_error(BEM_ERR_ARG, "unknown flags for bem_adjoint_v");
        need_device(ctx);
        need_one_component(ctx);
        const bool dev = (flags & BEM_DEVICE_PTR) != 0;
        const int K = ctx->hgeo.K;
        const size_t bytes = (size_t)nrhs * ctx->freq.L * 3 * (size_t)K * sizeof(zd);
        hipStream_t st = ctx->stream;
        Staged sw, sx;
        stage_in(sw, w, bytes, dev, st);
        stage_in(sx, x, bytes, dev, st);
        DevBuf work;
        work.alloc(adjoint_work_doubles(K) * sizeof(double));
        double *sums = nullptr, *tiles = nullptr, *self_out = nullptr;
        int ntiles = 0;
        launch_adjoint_v(ctx->devctx(ctx->dgeo.geo, nullptr), nrhs, (const zd*)sw.dev, (const zd*)sx.dev, work.as<double>(),
                         &sums, &tiles, &ntiles, &self_out, st);
        // U is proportional to 1 / rho
        adjoint_finish(ctx, sums, tiles, ntiles, self_out, -1.0 / ctx->rho, value, grad_nodes, grad_mat);
        return BEM_OK;
    });
}

int bem_adjoint_k(bem_ctx* ctx, int32_t op, int32_t nrhs, const void* w, const void* x, int32_t flags, double* value,
                  double* grad_nodes, double* grad_mat)
{
    if (!ctx) return BEM_ERR_ARG;
    return guarded(ctx, [&]() -> int {
        need_state(ctx);
        if (op != BEM_OP_K && op != BEM_OP_HK) throw api_error(BEM_ERR_ARG, "bem_adjoint_k takes BEM_OP_K or BEM_OP_HK");
        if (nrhs < 1 || !w || !x) throw api_error(BEM_ERR_ARG, "need nrhs >= 1 and buffers");
        if (flags & ~BEM_DEVICE_PTR) throw api_error(BEM_ERR_ARG, "unknown flags for bem_adjoint_k");
        need_device(ctx);
        need_one_component(ctx);
        const bool dev = (flags & BEM_DEVICE_PTR) != 0;
        const int K = ctx->hgeo.K;
        const size_t bytes = (size_t)nrhs * ctx->freq.L * 3 * (size_t)K * sizeof(zd);
        hipStream_t st = ctx->stream;
        Staged sw, sx;
        stage_in(sw, w, bytes, dev, st);
        stage_in(sx, x, bytes, dev, st);
        DevBuf work;
        work.alloc(adjoint_work_doubles(K) * sizeof(double));
        double *sums = nullptr, *tiles = nullptr, *self_out = nullptr;
        int ntiles = 0;
        launch_adjoint_k(ctx->devctx(ctx->dgeo.geo, nullptr), op == BEM_OP_HK, nrhs, (const zd*)sw.dev, (const zd*)sx.dev,
                         work.as<double>(), &sums, &tiles, &ntiles, &self_out, st);
        // T does not depend on rho
        adjoint_finish(ctx, sums, tiles, ntiles, self_out, 0.0, value, grad_nodes, grad_mat);
        return BEM_OK;
    });
}

struct bem_batch {
    bem_ctx* ctx = nullptr;
    std::vector<bem_op*> ops;
    bem::BatchPlan* plan = nullptr;
    ~bem_batch()
    {
        if (plan) bem::batch_destroy(plan);
        for (bem_op* o : ops) o->batches--;
    }
};

int bem_batch_create(bem_op* const* ops, int32_t nops, int32_t nrhs, int32_t flags, bem_batch** out)
{
    if (!ops || !out || nops < 1 || !ops[0]) return BEM_ERR_ARG;
    bem_ctx* ctx = ops[0]->ctx;
    return guarded(ctx, [&]() -> int {
        *out = nullptr;
        if (nops > 16) throw api_error(BEM_ERR_ARG, "at most 16 operators per batch");
        if (nrhs < 1) throw api_error(BEM_ERR_ARG, "need nrhs >= 1");
        if (flags & ~(BEM_BATCH_GRAPH | BEM_BATCH_TUNE)) throw api_error(BEM_ERR_ARG, "unknown batch flags");
        need_device(ctx);
        for (int o = 0; o < nops; ++o) {
            const bem_op* op = ops[o];
            if (!op || op->kind != 1) throw api_error(BEM_ERR_ARG, "batch of compressed operators only");
            if (op->L != ops[0]->L) throw api_error(BEM_ERR_ARG, "operators of a batch need the same L");
            if (op->ctx->device != ctx->device) throw api_error(BEM_ERR_ARG, "operators on different devices");
            for (int q = 0; q < o; ++q)
                if (ops[q] == op) throw api_error(BEM_ERR_ARG, "operator listed twice");
        }
        if ((size_t)nrhs * ops[0]->L > (1u << 20)) throw api_error(BEM_ERR_ARG, "nrhs * L above 2^20");
        auto b = std::make_unique<bem_batch>();
        b->ctx = ctx;
        b->plan = bem::batch_create(ops, nops, nrhs, flags, ctx->stream);
        b->ops.assign(ops, ops + nops);
        for (bem_op* o : b->ops) o->batches++;
        *out = b.release();
        return BEM_OK;
    });
}

int bem_batch_apply(bem_batch* b, const void* const* x, void* const* y, int32_t flags)
{
    if (!b) return BEM_ERR_ARG;
    bem_ctx* ctx = b->ctx;
    return guarded(ctx, [&]() -> int {
        if (!x || !y) throw api_error(BEM_ERR_ARG, "need buffers");
        const int n = (int)b->ops.size();
        for (int o = 0; o < n; ++o)
            if (!x[o] || !y[o]) throw api_error(BEM_ERR_ARG, "null buffer in the batch");
        if (flags & ~BEM_DEVICE_PTR) throw api_error(BEM_ERR_ARG, "unknown flags for bem_batch_apply");
        const bool dev = (flags & BEM_DEVICE_PTR) != 0;
        bem_batch_info info{};
        bem::batch_info(b->plan, &info);
        if (info.graph && !dev) throw api_error(BEM_ERR_ARG, "a graph batch takes device buffers");
        need_device(ctx);
        hipStream_t st = ctx->stream;
        std::vector<Staged> sx(n), sy(n);
        std::vector<const zd*> xd(n);
        std::vector<zd*> yd(n);
        std::vector<size_t> bytes(n);
        for (int o = 0; o < n; ++o) {
            bytes[o] = (size_t)info.nrhs * info.L * 3 * (size_t)b->ops[o]->K * sizeof(zd);
            stage_in(sx[o], x[o], bytes[o], dev, st);
            stage_out(sy[o], y[o], bytes[o], dev);
            xd[o] = (const zd*)sx[o].dev;
            yd[o] = (zd*)sy[o].dev;
        }
        bem::batch_apply(b->plan, xd.data(), yd.data(), st);
        for (int o = 0; o < n; ++o) finish_out(sy[o], y[o], bytes[o], dev, st);
        return BEM_OK;
    });
}

int bem_batch_info_get(const bem_batch* b, bem_batch_info* info)
{
    if (!b || !info) return BEM_ERR_ARG;
    bem::batch_info(b->plan, info);
    return BEM_OK;
}

int bem_batch_destroy(bem_batch* b)
{
    if (!b) return BEM_ERR_ARG;
    if (b->ctx && b->ctx->device >= 0) (void)hipSetDevice(b->ctx->device);
    delete b;
    return BEM_OK;
}

int bem_op_destroy(bem_op* op)
{
    if (!op) return BEM_ERR_ARG;
    if (op->batches > 0) return fail(op->ctx, BEM_ERR_STATE, "a batch still uses this operator");
    if (op->ctx && op->ctx->device >= 0) (void)hipSetDevice(op->ctx->device);
    delete op;
    return BEM_OK;
}

}  // extern "C"
