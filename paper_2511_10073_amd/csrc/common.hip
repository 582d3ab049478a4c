// Errors, the stream-ordered allocator and the integer prefix scan.
#include <mutex>

#include "ahr_internal.hpp"
#include "device_util.hpp"

namespace ahr {

static thread_local std::string t_last_error;

void set_error(ahr_status, const std::string& msg) { t_last_error = msg; }

std::string& last_error_ref() { return t_last_error; }

ahr_status fail(ahr_status code, const std::string& msg) {
    set_error(code, msg);
    return code;
}

void hip_check(hipError_t e, const char* what, const char* file, int line) {
    if (e == hipSuccess) return;
    char buf[512];
    snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    ahr_status code = (e == hipErrorOutOfMemory) ? AHR_ENOMEM : AHR_EDEVICE;
    throw Error{code, buf};
}

// ---------------------------------------------------------------- allocator

static std::once_flag g_pool_once[64];

static void prepare_pool(int dev) {
    // Keep freed blocks in the device's default pool so repeated graph
    // builds reuse memory instead of returning it to the driver.
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    (void)hipGetLastError();
}

void* dev_alloc(size_t bytes, hipStream_t s) {
    int dev = 0;
    AHR_HIP(hipGetDevice(&dev));
    if (dev >= 0 && dev < 64) std::call_once(g_pool_once[dev], prepare_pool, dev);
    void* p = nullptr;
    size_t b = bytes ? bytes : 1;
    b = (b + 255) & ~size_t(255);
    hipError_t e = hipMallocAsync(&p, b, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        char buf[160];
        snprintf(buf, sizeof buf, "device allocation of %zu bytes failed: %s", b, hipGetErrorString(e));
        throw Error{AHR_ENOMEM, buf};
    }
    return p;
}

void dev_free(void* p, hipStream_t s) {
    if (p) (void)hipFreeAsync(p, s);
}

// ---------------------------------------------------------------- scan

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

size_t scan_tmp_elems(int64_t n) { return static_cast<size_t>((n + kScanTile - 1) / kScanTile) + 2; }

template <class Tin>
__global__ void __launch_bounds__(kScanThreads) k_tile_sums(const Tin* __restrict__ in, int64_t n,
                                                            int64_t* __restrict__ sums) {
    __shared__ int64_t red[kScanThreads / 64];
    int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
    int64_t v = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + static_cast<int64_t>(k) * kScanThreads + threadIdx.x;
        if (i < n) v += static_cast<int64_t>(in[i]);
    }
    v = block_sum_i64<kScanThreads>(v, red);
    if (threadIdx.x == 0) sums[blockIdx.x] = v;
}

// Exclusive scan of the tile sums by one block; sums[ntiles] = total.
__global__ void __launch_bounds__(1024) k_scan_sums(int64_t* __restrict__ sums, int64_t ntiles) {
    __shared__ int64_t red[1024 / 64];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b = 0; b < ntiles; b += 1024) {
        int64_t i = b + threadIdx.x;
        int64_t v = i < ntiles ? sums[i] : 0;
        int64_t tot;
        int64_t ex = block_exclusive_scan_i64<1024>(v, red, &tot);
        int64_t c = carry;
        __syncthreads();
        if (i < ntiles) sums[i] = c + ex;
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[ntiles] = carry;
}

template <class Tin, class Tout>
__global__ void __launch_bounds__(kScanThreads) k_tile_scan(const Tin* __restrict__ in, int64_t n,
                                                            const int64_t* __restrict__ sums,
                                                            int64_t ntiles, Tout* __restrict__ out) {
    __shared__ int64_t red[kScanThreads / 64];
    int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + static_cast<int64_t>(threadIdx.x) * kScanItems;
    int64_t v[kScanItems];
    int64_t local = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        v[k] = i < n ? static_cast<int64_t>(in[i]) : 0;
        local += v[k];
    }
    int64_t tot;
    int64_t ex = block_exclusive_scan_i64<kScanThreads>(local, red, &tot);
    int64_t run = sums[blockIdx.x] + ex;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = static_cast<Tout>(run);
        run += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = static_cast<Tout>(sums[ntiles]);
}

template <class Tin, class Tout>
static void scan_impl(const Tin* in, Tout* out, int64_t n, int64_t* tmp, hipStream_t s) {
    int64_t ntiles = (n + kScanTile - 1) / kScanTile;   // n > 0
    hipLaunchKernelGGL((k_tile_sums<Tin>), dim3(ntiles), dim3(kScanThreads), 0, s, in, n, tmp);
    AHR_LAUNCHED("k_tile_sums");
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, tmp, ntiles);
    AHR_LAUNCHED("k_scan_sums");
    hipLaunchKernelGGL((k_tile_scan<Tin, Tout>), dim3(ntiles), dim3(kScanThreads), 0, s, in, n, tmp, ntiles, out);
    AHR_LAUNCHED("k_tile_scan");
}

void scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s) {
    if (n == 0) {
        AHR_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), s));
        return;
    }
    scan_impl<int32_t, int64_t>(in, out, n, tmp, s);
}

void scan_i32_to_i32(const int32_t* in, int32_t* out, int64_t n, int64_t* tmp, hipStream_t s) {
    if (n == 0) {
        AHR_HIP(hipMemsetAsync(out, 0, sizeof(int32_t), s));
        return;
    }
    scan_impl<int32_t, int32_t>(in, out, n, tmp, s);
}

// ---------------------------------------------------------------- lists, fills

__global__ void k_list_rows(const int32_t* __restrict__ flag, const int32_t* __restrict__ rank, int32_t n,
                            int32_t* __restrict__ list) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n && flag[i]) list[rank[i]] = static_cast<int32_t>(i);
}

void list_rows(const int32_t* flags, const int32_t* rank, int32_t n, int32_t* list, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_list_rows, dim3(grid_for(n, 256)), dim3(256), 0, s, flags, rank, n, list);
    AHR_LAUNCHED("k_list_rows");
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

void fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    AHR_LAUNCHED("k_fill_i32");
}

}  // namespace ahr
