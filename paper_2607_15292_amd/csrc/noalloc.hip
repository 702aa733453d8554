// noalloc.hip -- the per-slice ACA + recompression of one matrix (the bem_aca_matrix pass)
// on device buffers, with no device or host allocation: for callers that cannot allocate
// (code under HIP graph capture, serving loops, harnesses that forbid hipMalloc).
//
// The copy of the input matrix (the recompression writes the factors over it), the ACA
// columns, the recompression matrices and the two result counts live in `scratch`, one
// file-scope device array of NOALLOC_SCRATCH_BYTES.  Each GPU the library runs on holds its
// own copy until the process ends; its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and kept in `g_scratch`.  Host code never
// passes the array's name to a kernel or a copy: on the host that name is only a stand-in,
// not a device address.  Every call on one GPU shares its array, so calls that overlap on
// one GPU (several streams or threads) race.  Nothing in the array has to start at zero:
// the ACA kernels initialise what they read (used-row flags, tolerance, column count).
#include <algorithm>
#include <cstdint>
#include <mutex>

#include "../../include/bem.h"
#include "aca3d.hpp"
#include "host.hpp"

static __device__ __align__(256) char scratch[BEM_ACA_NOALLOC_SCRATCH_BYTES];

namespace bem {

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = BEM_ACA_NOALLOC_SCRATCH_BYTES;
constexpr int NOALLOC_MAX = BEM_ACA_NOALLOC_MAX_ELEMENTS;
constexpr int NOALLOC_KMAX = 96;  // the ACA column capacity of bem_aca_matrix
// layout: [matrix copy | ACA scratch | 2 result ints], each part 256-byte aligned
constexpr size_t H_BYTES = (size_t)9 * NOALLOC_MAX * NOALLOC_MAX * 16;

constexpr int MAX_DEVICES = 64;
std::mutex g_mutex;
char* g_scratch[MAX_DEVICES] = {};

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// res = (ACA columns, rank) from the ACA kernels; the factors Ubar (3m x kk) then Vbar
// (3n x kk), row-major, sit at the start of H.  Copies them to U, V and the counts to kckk.
__global__ __launch_bounds__(256) void k_noalloc_out(const char* H, const int* res, int m, int n, int esize,
                                                     char* U, char* V, int* kckk)
{
    const int kk = res[1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        kckk[0] = res[0];
        kckk[1] = kk;
    }
    if (kk <= 0) return;
    const size_t nu = (size_t)3 * m * kk * esize / 8, nv = (size_t)3 * n * kk * esize / 8;  // 8-byte words
    const unsigned long long* src = (const unsigned long long*)H;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < nu + nv; q += (size_t)gridDim.x * blockDim.x) {
        const unsigned long long w = src[q];
        if (q < nu) ((unsigned long long*)U)[q] = w;
        else ((unsigned long long*)V)[q - nu] = w;
    }
}

bool is_device_ptr(const void* p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

}  // namespace

// Device address of `scratch` on `device` (current): looked up once per device.
char* noalloc_scratch(int device)
{
    if (device < 0 || device >= MAX_DEVICES) throw ApiError(BEM_ERR_ARG, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[device]) {
        void* ptr = nullptr;
        BEM_HIP_TRY(hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)));
        g_scratch[device] = (char*)ptr;
    }
    return g_scratch[device];
}

void aca_matrix_noalloc_impl(int device, bool fp32, int m, int n, const void* A, double tol, int max_cols,
                             int32_t* kckk, void* U, void* V, hipStream_t st)
{
    if (m > NOALLOC_MAX || n > NOALLOC_MAX)
        throw ApiError(BEM_ERR_ARG, "bem_aca_matrix_noalloc: m and n must not exceed BEM_ACA_NOALLOC_MAX_ELEMENTS");
    const size_t es = fp32 ? 8 : 16;
    if (((uintptr_t)A | (uintptr_t)U | (uintptr_t)V) % es != 0 || (uintptr_t)kckk % 4 != 0)
        throw ApiError(BEM_ERR_ARG, "bem_aca_matrix_noalloc: misaligned buffer");
    if (!is_device_ptr(A) || !is_device_ptr(U) || !is_device_ptr(V) || !is_device_ptr(kckk))
        throw ApiError(BEM_ERR_ARG, "bem_aca_matrix_noalloc: buffers must be device memory");
    int cap = max_cols > 0 ? max_cols : face_aca_cap(m, n);
    cap = std::min(std::min(cap, 3 * std::min(m, n)), NOALLOC_KMAX);
    cap -= cap % 3;
    const int kmax = std::max(cap, 3);
    const size_t sbytes = align256(aca_scratch_doubles(m, n, kmax) * sizeof(double));
    if (H_BYTES + sbytes + 256 > NOALLOC_SCRATCH_BYTES)
        throw ApiError(BEM_ERR_ARG, "bem_aca_matrix_noalloc: scratch layout exceeds its size");
    char* base = noalloc_scratch(device);
    char* H = base;
    double* work = (double*)(base + H_BYTES);
    int* res = (int*)(base + H_BYTES + sbytes);
    BEM_HIP_TRY(hipMemcpyAsync(H, A, es * 9 * (size_t)m * n, hipMemcpyDeviceToDevice, st));
    launch_aca_matrix(H, m, n, fp32 ? 1 : 0, tol, cap, kmax, work, res, st);
    hipLaunchKernelGGL(k_noalloc_out, dim3(64), dim3(256), 0, st, (const char*)H, (const int*)res, m, n, (int)es,
                       (char*)U, (char*)V, (int*)kckk);
    BEM_HIP_TRY(hipGetLastError());
}

}  // namespace bem
