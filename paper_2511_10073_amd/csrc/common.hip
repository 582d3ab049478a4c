// Errors, the stream-ordered allocator and the integer prefix scan.
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>

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
//
// A caching allocator: freed device blocks are kept (per device, by size
// class) and handed out again, so the graph builds of an initializer loop
// allocate from the driver only the first time.  A block reused on the
// stream it was freed on needs nothing more.  A block reused on another
// stream is ordered behind its free by an event wait.  Each event record
// costs the GPU a few microseconds of queue processing, so frees do not
// record one each: at the end of every entry point (flush_frees), one event
// per stream covers all the blocks freed on it during the call.  A block
// that another stream takes before that gets its stream's event at once.
// The events are recycled through a per-device pool.
// ahr_memory_trim() returns the cache to the driver.

namespace {

// An event recorded after the frees of one stream; the blocks it covers
// share it and the last one reused returns it to the pool.
struct FreeEvent {
    hipEvent_t e;       // null: the frees are known to be complete
    int refs;
    int device;
};

struct Block {
    void* p;
    size_t bytes;
    hipStream_t stream;
    FreeEvent* done;    // null while the free is pending (no event yet)
    int device;
};

std::mutex g_alloc_mu;
std::multimap<size_t, Block> g_free;                  // by size class
std::unordered_map<void*, std::pair<size_t, int>> g_live;   // ptr -> (size class, device)
std::unordered_map<int, std::vector<hipEvent_t>> g_events;  // idle events per device

// All under g_alloc_mu.  take_event returns null if no event can be made.
hipEvent_t take_event(int dev) {
    auto& v = g_events[dev];
    if (!v.empty()) {
        hipEvent_t e = v.back();
        v.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

void drop_ref(FreeEvent* fe) {
    if (!fe || --fe->refs > 0) return;
    if (fe->e) g_events[fe->device].push_back(fe->e);
    delete fe;
}

// One event on (device, stream) for every pending block freed there; if
// no event can be recorded, wait for the stream instead.
void flush_stream_locked(int dev, hipStream_t s) {
    auto* fe = new FreeEvent{take_event(dev), 0, dev};
    if (!fe->e || hipEventRecord(fe->e, s) != hipSuccess) {
        (void)hipGetLastError();
        if (fe->e) g_events[dev].push_back(fe->e);
        fe->e = nullptr;
        (void)hipStreamSynchronize(s);
    }
    for (auto& kv : g_free) {
        Block& b = kv.second;
        if (!b.done && b.device == dev && b.stream == s) {
            b.done = fe;
            ++fe->refs;
        }
    }
    if (fe->refs == 0) {
        fe->refs = 1;
        drop_ref(fe);
    }
}

void flush_all_locked() {
    for (;;) {
        const Block* pending = nullptr;
        for (auto& kv : g_free)
            if (!kv.second.done) {
                pending = &kv.second;
                break;
            }
        if (!pending) return;
        int cur = 0;
        (void)hipGetDevice(&cur);
        if (pending->device != cur) (void)hipSetDevice(pending->device);
        flush_stream_locked(pending->device, pending->stream);
        if (pending->device != cur) (void)hipSetDevice(cur);
    }
}

size_t size_class(size_t b) {
    b = b < 256 ? 256 : b;
    if (b <= (size_t(1) << 20)) {
        size_t c = 256;
        while (c < b) c <<= 1;
        return c;
    }
    const size_t mib = size_t(1) << 20;
    size_t c = (b + mib - 1) / mib * mib;
    // round large blocks up to 1/8 steps of their power of two to bound the classes
    size_t top = mib;
    while (top < c) top <<= 1;
    size_t step = top / 8 > mib ? top / 8 : mib;
    return (c + step - 1) / step * step;
}

}  // namespace

// ---------------------------------------------------------------- arenas

struct Arena {
    char* base;
    size_t size;
    std::map<size_t, size_t> free_blocks;            // offset -> length
    std::unordered_map<size_t, size_t> live;         // offset -> length
    std::map<size_t, hipStream_t> freed_on;          // offset of a free block -> stream of its last free
    size_t used = 0, peak = 0;
};

namespace {
std::vector<Arena*> g_arenas;                        // under g_alloc_mu
thread_local Arena* t_arena = nullptr;

constexpr size_t kArenaAlign = 256;

void* arena_alloc(Arena& a, size_t bytes, hipStream_t s) {
    const size_t need = (bytes < 1 ? 1 : bytes + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
    for (auto it = a.free_blocks.begin(); it != a.free_blocks.end(); ++it) {
        if (it->second < need) continue;
        const size_t off = it->first, len = it->second;
        a.free_blocks.erase(it);
        if (len > need) a.free_blocks[off + need] = len - need;
        auto fs = a.freed_on.find(off);
        if (fs != a.freed_on.end()) {
            // freed on another stream: its last work there must be done
            if (fs->second != s) AHR_HIP(hipStreamSynchronize(fs->second));
            a.freed_on.erase(fs);
        }
        a.live[off] = need;
        a.used += need;
        if (a.used > a.peak) a.peak = a.used;
        return a.base + off;
    }
    char buf[200];
    snprintf(buf, sizeof buf,
             "workspace too small: %zu more bytes needed with %zu of %zu in use (ask ahr_graph_workspace_size)",
             need, a.used, a.size);
    throw Error{AHR_ENOMEM, buf};
}

void arena_free(Arena& a, void* p, hipStream_t s) {
    const size_t off = static_cast<size_t>(static_cast<char*>(p) - a.base);
    auto it = a.live.find(off);
    if (it == a.live.end()) return;
    size_t start = off, len = it->second;
    a.used -= len;
    a.live.erase(it);
    // the merged block remembers the stream of this free (the latest one)
    auto nx = a.free_blocks.find(off + len);
    if (nx != a.free_blocks.end()) {
        len += nx->second;
        a.freed_on.erase(nx->first);
        a.free_blocks.erase(nx);
    }
    auto pv = a.free_blocks.lower_bound(off);
    if (pv != a.free_blocks.begin()) {
        --pv;
        if (pv->first + pv->second == off) {
            start = pv->first;
            len += pv->second;
            a.freed_on.erase(pv->first);
            a.free_blocks.erase(pv);
        }
    }
    a.free_blocks[start] = len;
    a.freed_on[start] = s;
}
}  // namespace

Arena* arena_create(void* base, size_t bytes) {
    auto* a = new Arena();
    const auto b = reinterpret_cast<uintptr_t>(base);
    const uintptr_t aligned = (b + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
    const size_t skip = static_cast<size_t>(aligned - b);
    a->base = reinterpret_cast<char*>(aligned);
    a->size = bytes > skip ? (bytes - skip) / kArenaAlign * kArenaAlign : 0;
    if (a->size) a->free_blocks[0] = a->size;
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_arenas.push_back(a);
    return a;
}

void arena_destroy(Arena* a) noexcept {
    if (!a) return;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        for (size_t i = 0; i < g_arenas.size(); ++i)
            if (g_arenas[i] == a) {
                g_arenas.erase(g_arenas.begin() + static_cast<long>(i));
                break;
            }
    }
    delete a;
}

size_t arena_peak(const Arena* a) { return a ? a->peak : 0; }
size_t arena_size(const Arena* a) { return a ? a->size : 0; }

ArenaScope::ArenaScope(Arena* a) : prev_(t_arena) { t_arena = a; }
ArenaScope::~ArenaScope() { t_arena = prev_; }

void* dev_alloc(size_t bytes, hipStream_t s) {
    if (t_arena) {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        return arena_alloc(*t_arena, bytes, s);
    }
    int dev = 0;
    AHR_HIP(hipGetDevice(&dev));
    const size_t cls = size_class(bytes);
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        // a block freed on this stream first (no wait), else any
        auto pick = g_free.end();
        for (auto it = g_free.lower_bound(cls); it != g_free.end() && it->first == cls; ++it) {
            if (it->second.device != dev) continue;
            if (pick == g_free.end()) pick = it;
            if (it->second.stream == s) {
                pick = it;
                break;
            }
        }
        if (pick != g_free.end()) {
            if (pick->second.stream != s) {
                if (!pick->second.done) flush_stream_locked(dev, pick->second.stream);
                if (pick->second.done->e) AHR_HIP(hipStreamWaitEvent(s, pick->second.done->e, 0));
            }
            Block b = pick->second;
            g_free.erase(pick);
            drop_ref(b.done);
            g_live[b.p] = {cls, dev};
            return b.p;
        }
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, cls);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        ahr_memory_trim();
        e = hipMalloc(&p, cls);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        char buf[160];
        snprintf(buf, sizeof buf, "device allocation of %zu bytes failed: %s", cls, hipGetErrorString(e));
        throw Error{AHR_ENOMEM, buf};
    }
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_live[p] = {cls, dev};
    return p;
}

void dev_free(void* p, hipStream_t s) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    for (Arena* a : g_arenas) {
        if (static_cast<char*>(p) >= a->base && static_cast<char*>(p) < a->base + a->size) {
            arena_free(*a, p, s);
            return;
        }
    }
    auto it = g_live.find(p);
    if (it == g_live.end()) return;
    g_free.emplace(it->second.first, Block{p, it->second.first, s, nullptr, it->second.second});
    g_live.erase(it);
}

void flush_frees() noexcept {
    try {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        flush_all_locked();
    } catch (...) {
    }
}

hipStream_t side_stream() {
    static std::mutex mu;
    static std::unordered_map<int, hipStream_t> streams;
    int dev = 0;
    AHR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = streams.find(dev);
    if (it != streams.end()) return it->second;
    hipStream_t st = nullptr;
    AHR_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    streams[dev] = st;
    return st;
}

// ---------------------------------------------------------------- scan

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

size_t scan_tmp_elems(int64_t n) { return static_cast<size_t>((n + kScanTile - 1) / kScanTile) + 2; }

// Loads here are unconditional, indexes clamped to the last element and the
// values masked afterwards: a load under a per-lane branch is waited for
// where the branch joins, which would run the loads one after another.

template <class Tin>
__global__ void __launch_bounds__(kScanThreads) k_tile_sums(const Tin* __restrict__ in, int64_t n,
                                                            int64_t* __restrict__ sums) {
    __shared__ int64_t red[kScanThreads / 64];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x;
    Tin x[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + static_cast<int64_t>(k) * kScanThreads;
        x[k] = in[i < n ? i : n - 1];
    }
    int64_t v = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        v += base + static_cast<int64_t>(k) * kScanThreads < n ? static_cast<int64_t>(x[k]) : 0;
    v = block_sum_i64<kScanThreads>(v, red);
    if (threadIdx.x == 0) sums[blockIdx.x] = v;
}

// The kScanItems elements of thread t of a tile (t kScanItems onwards), as
// int64, zero past n.  With V (16-byte aligned int32 input), a thread whose
// items all lie below n reads them as two 16-byte loads.
template <bool V, class Tin>
__device__ __forceinline__ int64_t load_items(const Tin* __restrict__ in, int64_t n, int64_t base, int64_t* v) {
    if constexpr (V && sizeof(Tin) == 4) {
        static_assert(kScanItems == 8, "two 16-byte loads per thread");
        if (base + kScanItems <= n) {
            const int4* p = reinterpret_cast<const int4*>(in + base);
            const int4 a = p[0], b = p[1];
            v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w;
            v[4] = b.x, v[5] = b.y, v[6] = b.z, v[7] = b.w;
            return v[0] + v[1] + v[2] + v[3] + v[4] + v[5] + v[6] + v[7];
        }
    }
    Tin x[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) x[k] = in[base + k < n ? base + k : n - 1];
    int64_t local = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? static_cast<int64_t>(x[k]) : 0;
        local += v[k];
    }
    return local;
}

// out[base + k] = run + v[0] + ... + v[k-1] for the items below n; with V
// (16-byte aligned output) a thread whose items all lie below n writes them
// with 16-byte stores.
template <bool V, class Tout>
__device__ __forceinline__ void store_items(Tout* __restrict__ out, int64_t n, int64_t base, int64_t run,
                                            const int64_t* v) {
    Tout o[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        o[k] = static_cast<Tout>(run);
        run += v[k];
    }
    if constexpr (V) {
        if (base + kScanItems <= n) {
            int4* p = reinterpret_cast<int4*>(out + base);
            constexpr int kVecs = kScanItems * sizeof(Tout) / sizeof(int4);
#pragma unroll
            for (int q = 0; q < kVecs; ++q) {
                int4 w;
                __builtin_memcpy(&w, reinterpret_cast<const char*>(o) + q * sizeof(int4), sizeof(int4));
                p[q] = w;
            }
            return;
        }
    }
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) out[base + k] = o[k];
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

template <bool V, class Tin, class Tout>
__global__ void __launch_bounds__(kScanThreads) k_tile_scan(const Tin* __restrict__ in, int64_t n,
                                                            const int64_t* __restrict__ sums,
                                                            int64_t ntiles, Tout* __restrict__ out) {
    __shared__ int64_t red[kScanThreads / 64];
    int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + static_cast<int64_t>(threadIdx.x) * kScanItems;
    int64_t v[kScanItems];
    const int64_t local = load_items<V>(in, n, base, v);
    int64_t tot;
    int64_t ex = block_exclusive_scan_i64<kScanThreads>(local, red, &tot);
    store_items<V>(out, n, base, sums[blockIdx.x] + ex, v);
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = static_cast<Tout>(sums[ntiles]);
}

// Up to kDirectTiles tiles, the tile offsets are not scanned by a separate
// kernel: each workgroup of the final pass adds up the sums of the tiles
// before it (a few KB of cached reads), and workgroup 0 adds all of them for
// the total.
constexpr int64_t kDirectTiles = 4096;

template <bool V, class Tin, class Tout>
__global__ void __launch_bounds__(kScanThreads) k_tile_scan_direct(const Tin* __restrict__ in, int64_t n,
                                                                   int64_t* __restrict__ sums, int64_t ntiles,
                                                                   Tout* __restrict__ out) {
    __shared__ int64_t red[kScanThreads / 64];
    const int64_t upto = blockIdx.x == 0 ? ntiles : static_cast<int64_t>(blockIdx.x);   // >= 1
    int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + static_cast<int64_t>(threadIdx.x) * kScanItems;
    int64_t v[kScanItems];
    const int64_t local = load_items<V>(in, n, base, v);
    constexpr int U = 8;
    int64_t pre = 0;
    for (int64_t j0 = threadIdx.x; j0 < upto; j0 += U * kScanThreads) {
        int64_t t[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = j0 + u * kScanThreads;
            t[u] = sums[j < upto ? j : upto - 1];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) pre += j0 + u * kScanThreads < upto ? t[u] : 0;
    }
    pre = block_sum_i64<kScanThreads>(pre, red);
    const int64_t tile_off = blockIdx.x == 0 ? 0 : pre;
    int64_t tot;
    int64_t ex = block_exclusive_scan_i64<kScanThreads>(local, red, &tot);
    store_items<V>(out, n, base, tile_off + ex, v);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sums[ntiles] = pre;
        out[n] = static_cast<Tout>(pre);
    }
}

template <bool V, class Tin, class Tout>
static void scan_launch(const Tin* in, Tout* out, int64_t n, int64_t* tmp, int64_t ntiles, hipStream_t s) {
    if (ntiles <= kDirectTiles) {
        hipLaunchKernelGGL((k_tile_scan_direct<V, Tin, Tout>), dim3(ntiles), dim3(kScanThreads), 0, s, in, n, tmp,
                           ntiles, out);
        AHR_LAUNCHED("k_tile_scan_direct");
        return;
    }
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, tmp, ntiles);
    AHR_LAUNCHED("k_scan_sums");
    hipLaunchKernelGGL((k_tile_scan<V, Tin, Tout>), dim3(ntiles), dim3(kScanThreads), 0, s, in, n, tmp, ntiles, out);
    AHR_LAUNCHED("k_tile_scan");
}

template <class Tin, class Tout>
static void scan_impl(const Tin* in, Tout* out, int64_t n, int64_t* tmp, hipStream_t s) {
    int64_t ntiles = (n + kScanTile - 1) / kScanTile;   // n > 0
    hipLaunchKernelGGL((k_tile_sums<Tin>), dim3(ntiles), dim3(kScanThreads), 0, s, in, n, tmp);
    AHR_LAUNCHED("k_tile_sums");
    // 16-byte accesses when both arrays allow them (the offsets inside a
    // tile are multiples of 32 bytes)
    const bool vec = (reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) % 16 == 0;
    if (vec)
        scan_launch<true>(in, out, n, tmp, ntiles, s);
    else
        scan_launch<false>(in, out, n, tmp, ntiles, s);
}

void scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s) {
    if (n == 0) {
        AHR_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), s));
        return;
    }
    scan_impl<int32_t, int64_t>(in, out, n, tmp, s);
}

__global__ void k_zero_i64(int64_t* p) { *p = 0; }

const int64_t* scan_i32_total(const int32_t* in, int32_t* out, int64_t n, int64_t* tmp, hipStream_t s) {
    if (n == 0) {
        AHR_HIP(hipMemsetAsync(out, 0, sizeof(int32_t), s));
        hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(1), 0, s, tmp);
        AHR_LAUNCHED("k_zero_i64");
        return tmp;
    }
    scan_impl<int32_t, int32_t>(in, out, n, tmp, s);
    return tmp + (n + kScanTile - 1) / kScanTile;
}

int64_t scan_i32_checked(const int32_t* in, int32_t* out, int64_t n, int64_t* tmp, hipStream_t s) {
    if (n == 0) {
        AHR_HIP(hipMemsetAsync(out, 0, sizeof(int32_t), s));
        return 0;
    }
    scan_impl<int32_t, int32_t>(in, out, n, tmp, s);
    int64_t ntiles = (n + kScanTile - 1) / kScanTile;
    return read_i64(tmp + ntiles, s);
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

struct PtrPack {
    const void* p[12];
    int wide[12];   // 8-byte source word
};

// Small reads go straight into pinned, coherent host memory: one gather
// kernel and one stream synchronisation, no copy.
__global__ void k_gather_scalars(PtrPack src, int n, int64_t* dst) {
    int i = threadIdx.x;
    if (i < n)
        dst[i] = src.wide[i] ? *static_cast<const int64_t*>(src.p[i])
                             : static_cast<int64_t>(*static_cast<const int32_t*>(src.p[i]));
}

namespace {

// 20 pinned words per device and host thread: 0..7 for synchronous reads,
// 8..19 for the split read.
int64_t* host_words(int dev) {
    static thread_local int64_t* buf[64] = {nullptr};
    if (dev < 0 || dev >= 64) throw Error{AHR_EDEVICE, "device ordinal out of range"};
    if (!buf[dev]) AHR_HIP(hipHostMalloc(reinterpret_cast<void**>(&buf[dev]), 20 * sizeof(int64_t),
                                         hipHostMallocCoherent));
    return buf[dev];
}

struct SplitRead {
    int dev = -1;
    hipEvent_t ev = nullptr;
    int n = 0;
};
thread_local SplitRead g_split;

void read_words(const PtrPack& pk, int n, int64_t* out, hipStream_t s) {
    int dev = 0;
    AHR_HIP(hipGetDevice(&dev));
    int64_t* hw = host_words(dev);
    hipLaunchKernelGGL(k_gather_scalars, dim3(1), dim3(64), 0, s, pk, n, hw);
    AHR_LAUNCHED("k_gather_scalars");
    AHR_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < n; ++k) out[k] = hw[k];
}

}  // namespace

void read_scalars_begin(const std::vector<const int32_t*>& src, hipStream_t s) {
    if (src.size() > 12) throw Error{AHR_EDEVICE, "read_scalars_begin: at most 12"};
    int dev = 0;
    AHR_HIP(hipGetDevice(&dev));
    if (g_split.ev && g_split.dev != dev) {
        AHR_HIP(hipEventDestroy(g_split.ev));
        g_split.ev = nullptr;
    }
    if (!g_split.ev)     // a system-scope release: the host reads what the gather wrote
        AHR_HIP(hipEventCreateWithFlags(&g_split.ev, hipEventDisableTiming | hipEventReleaseToSystem));
    g_split.dev = dev;
    PtrPack pk{};
    for (size_t k = 0; k < src.size(); ++k) pk.p[k] = src[k];
    g_split.n = static_cast<int>(src.size());
    hipLaunchKernelGGL(k_gather_scalars, dim3(1), dim3(64), 0, s, pk, g_split.n, host_words(dev) + 8);
    AHR_LAUNCHED("k_gather_scalars");
    AHR_HIP(hipEventRecord(g_split.ev, s));
}

void read_scalars_end(int32_t* host, int n) {
    if (!g_split.ev || n > g_split.n) throw Error{AHR_EDEVICE, "read_scalars_end without its begin"};
    AHR_HIP(hipEventSynchronize(g_split.ev));
    const int64_t* hw = host_words(g_split.dev) + 8;
    for (int k = 0; k < n; ++k) host[k] = static_cast<int32_t>(hw[k]);
}

void read_words(std::initializer_list<DevWord> src, int64_t* out, hipStream_t s) {
    if (src.size() == 0) return;
    if (src.size() > 8) throw Error{AHR_EDEVICE, "read_words: at most 8"};
    PtrPack pk{};
    int k = 0;
    for (const DevWord& w : src) {
        pk.p[k] = w.p;
        pk.wide[k] = w.wide;
        ++k;
    }
    read_words(pk, k, out, s);
}

void read_scalars(const std::vector<const int32_t*>& src, int32_t* host, hipStream_t s) {
    if (src.empty()) return;
    if (src.size() > 8) throw Error{AHR_EDEVICE, "read_scalars: at most 8"};
    PtrPack pk{};
    for (size_t k = 0; k < src.size(); ++k) pk.p[k] = src[k];
    int64_t w[8];
    read_words(pk, static_cast<int>(src.size()), w, s);
    for (size_t k = 0; k < src.size(); ++k) host[k] = static_cast<int32_t>(w[k]);
}

int64_t read_i64(const int64_t* src, hipStream_t s) {
    PtrPack pk{};
    pk.p[0] = src;
    pk.wide[0] = 1;
    int64_t w = 0;
    read_words(pk, 1, &w, s);
    return w;
}

int32_t read_i32(const int32_t* src, hipStream_t s) {
    int32_t v = 0;
    read_scalars({src}, &v, s);
    return v;
}

double read_f64(const double* src, hipStream_t s) {
    const int64_t w = read_i64(reinterpret_cast<const int64_t*>(src), s);
    double d;
    std::memcpy(&d, &w, sizeof d);
    return d;
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

extern "C" ahr_status ahr_memory_trim(void) {
    std::lock_guard<std::mutex> lk(ahr::g_alloc_mu);
    ahr::flush_all_locked();
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : ahr::g_free) {
        ahr::Block& b = kv.second;
        if (b.done->e) (void)hipEventSynchronize(b.done->e);
        ahr::drop_ref(b.done);
        (void)hipSetDevice(b.device);
        (void)hipFree(b.p);
    }
    (void)hipSetDevice(cur);
    ahr::g_free.clear();
    for (auto& kv : ahr::g_events)
        for (hipEvent_t e : kv.second) (void)hipEventDestroy(e);
    ahr::g_events.clear();
    return AHR_OK;
}
