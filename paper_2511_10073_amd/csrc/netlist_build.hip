// Netlist part of the graph: macro pin expansion (Section V, "Macro pin
// expansion") and the clique/star net model with integer weights in units
// of 2^-32, merged into a canonical CSR (rows ascending, columns strictly
// ascending, parallel edges summed exactly).  Every structural step uses
// integer counts, scans and sorts, so the result is bit-identical from run
// to run and to any other exact implementation of the same definition.
#include <algorithm>

#include "ahr_internal.hpp"
#include "device_util.hpp"

namespace ahr {

namespace {

constexpr int kBT = 256;

// Device-side validation of the caller's netlist arrays.  bad[0] gets a
// nonzero code on the first violation found.
__global__ void k_validate(const int32_t* __restrict__ net_ptr, int32_t n_nets, const int32_t* __restrict__ pin_node,
                           int32_t n_pins, int32_t n_inst, int32_t* bad) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n_pins) {
        int v = pin_node[i];
        if (v < 0 || v >= n_inst) atomicCAS(bad, 0, 1);
    }
    if (i <= n_nets) {
        int a = net_ptr[i];
        if (i == 0 && a != 0) atomicCAS(bad, 0, 2);
        if (i == n_nets && a != n_pins) atomicCAS(bad, 0, 3);
        if (i < n_nets && net_ptr[i + 1] < a) atomicCAS(bad, 0, 4);
    }
}

__global__ void k_mark_mpin(const int32_t* __restrict__ pin_node, const uint8_t* __restrict__ flags, int32_t n_pins,
                            int32_t n_inst, int32_t expand, int32_t* __restrict__ is_mp) {
    int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= n_pins) return;
    const int v = pin_node[p];
    const uint8_t f = flags[v >= 0 && v < n_inst ? v : 0];      // clamped: runs before the netlist is verified
    is_mp[p] = (expand && (f & AHR_NODE_FIXED) && (f & AHR_NODE_MACRO)) ? 1 : 0;
}

__global__ void k_pin_nodes(const int32_t* __restrict__ pin_node, const int32_t* __restrict__ is_mp,
                            const int32_t* __restrict__ mp_rank, int32_t n_pins, int32_t n_inst,
                            int32_t* __restrict__ pin_node_x, int32_t* __restrict__ mp_owner,
                            int32_t* __restrict__ mp_pin) {
    int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= n_pins) return;
    int v = pin_node[p];
    if (is_mp[p]) {
        int r = mp_rank[p];
        pin_node_x[p] = n_inst + r;
        mp_owner[r] = v;
        mp_pin[r] = static_cast<int32_t>(p);
    } else {
        pin_node_x[p] = v;
    }
}

// Per net: star (more than clique_max pins), big (more pins than a wave),
// big star (a star whose spokes a whole workgroup averages).
__global__ void k_mark_star(const int32_t* __restrict__ net_ptr, int32_t n_nets, int32_t clique_max,
                            int32_t* __restrict__ is_star, int32_t* __restrict__ is_big,
                            int32_t* __restrict__ is_big_star) {
    int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n_nets) return;
    int deg = net_ptr[e + 1] - net_ptr[e];
    is_star[e] = deg > clique_max ? 1 : 0;
    is_big[e] = deg > kWave ? 1 : 0;
    is_big_star[e] = (deg > clique_max && deg > kStarMid) ? 1 : 0;
}

// Star index (rank among the stars) of every big-star net, ascending.
__global__ void k_list_big_stars(const int32_t* __restrict__ flag, const int32_t* __restrict__ rank,
                                 const int32_t* __restrict__ star_rank, int32_t n_nets, int32_t* __restrict__ out) {
    int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e < n_nets && flag[e]) out[rank[e]] = star_rank[e];
}

// Macro flags, and the count of movable macros in *movable.
__global__ void k_mark_macro(const uint8_t* __restrict__ flags, int32_t n, int32_t* __restrict__ out,
                             int32_t* __restrict__ movable) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint8_t f = flags[i];
    out[i] = (f & AHR_NODE_MACRO) ? 1 : 0;
    if ((f & AHR_NODE_MACRO) && !(f & AHR_NODE_FIXED)) atomicAdd(movable, 1);
}

// Net of every pin: one thread per net of at most a wave's worth of pins,
// one workgroup per bigger net (k_pin_net_big over the big-net list).
__global__ void k_pin_net(const int32_t* __restrict__ net_ptr, int32_t n_nets, int32_t* __restrict__ pin_net) {
    int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n_nets) return;
    const int lo = net_ptr[e], hi = net_ptr[e + 1];
    if (hi - lo > kWave) return;
    for (int p = lo; p < hi; ++p) pin_net[p] = static_cast<int32_t>(e);
}

__global__ void k_pin_net_big(const int32_t* __restrict__ big, const int32_t* __restrict__ net_ptr,
                              int32_t* __restrict__ pin_net) {
    const int e = big[blockIdx.x];
    for (int p = net_ptr[e] + threadIdx.x; p < net_ptr[e + 1]; p += blockDim.x) pin_net[p] = e;
}

// Integer weight of one clique pair / one star spoke (units of 2^-32),
// round-half-even of the float64 value, evaluated in this order:
//   clique: (2^32 w) / (p - 1)     star: ((2^32 w) p) / (p - 1)
__device__ __forceinline__ int64_t q_clique(float w, int p) {
    double wq = static_cast<double>(w) * 4294967296.0;
    return static_cast<int64_t>(__builtin_rint(wq / static_cast<double>(p - 1)));
}
__device__ __forceinline__ int64_t q_star(float w, int p) {
    double wq = static_cast<double>(w) * 4294967296.0;
    double num = wq * static_cast<double>(p);
    return static_cast<int64_t>(__builtin_rint(num / static_cast<double>(p - 1)));
}

// A raw (unsorted, unmerged) entry: column and integer weight, one 16-byte
// store per entry in the scatter and one load in the sorts.
struct alignas(16) RawEnt {
    int32_t col;
    int32_t pad;
    int64_t q;
};

__device__ __forceinline__ RawEnt raw_ent(int32_t col, int64_t q) {
    RawEnt e;
    e.col = col;
    e.pad = 0;
    e.q = q;
    return e;
}

struct NetArgs {
    const int32_t* net_ptr;
    const int32_t* pin_net;
    const int32_t* pin_x;
    const float* net_w;
    const int32_t* star_rank;
    int32_t n_nets, n_pins, clique_max, first_star;
};

// The nodes of the pins of a clique net of at most kNetUnroll pins, all
// loaded at once (indexes clamped to the last pin; a loop one load at a time
// would wait for each), and how many of them differ from v.
constexpr int kNetUnroll = 16;

__device__ __forceinline__ int clique_nodes(const int32_t* __restrict__ pin_x, int lo, int hi, int v, int* node) {
    int c = 0;
    if (hi - lo <= kNetUnroll) {
#pragma unroll
        for (int u = 0; u < kNetUnroll; ++u) node[u] = pin_x[lo + u < hi ? lo + u : hi - 1];
#pragma unroll
        for (int u = 0; u < kNetUnroll; ++u) c += (lo + u < hi && node[u] != v) ? 1 : 0;
    } else {
        for (int b = lo; b < hi; ++b) c += (pin_x[b] != v) ? 1 : 0;
    }
    return c;
}

// Entries each row receives (parallel edges counted separately).  Each pin
// reserves its run of its row's slots here, with the atomic that counts it:
// slot[p] = where the run starts inside the row (the run order inside a row
// does not matter: rows are sorted by column and equal columns merged by
// exact integer sums afterwards).
__global__ void k_row_counts(NetArgs a, int32_t* __restrict__ cnt, int32_t* __restrict__ slot) {
    int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= a.n_pins) return;
    int e = a.pin_net[p];
    int lo = a.net_ptr[e], hi = a.net_ptr[e + 1];
    int deg = hi - lo;
    if (deg < 2) return;
    int v = a.pin_x[p];
    if (deg <= a.clique_max) {
        int node[kNetUnroll];
        const int c = clique_nodes(a.pin_x, lo, hi, v, node);
        if (c) slot[p] = atomicAdd(&cnt[v], c);
    } else {
        slot[p] = atomicAdd(&cnt[v], 1);
        if (p == lo) cnt[a.first_star + a.star_rank[e]] = deg;
    }
}

// Raw entries: each pin writes its run at the slots it reserved while the
// rows were counted.
__global__ void k_scatter(NetArgs a, const int64_t* __restrict__ rp, const int32_t* __restrict__ slot,
                          RawEnt* __restrict__ raw) {
    int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= a.n_pins) return;
    int e = a.pin_net[p];
    int lo = a.net_ptr[e], hi = a.net_ptr[e + 1];
    int deg = hi - lo;
    if (deg < 2) return;
    int v = a.pin_x[p];
    float w = a.net_w ? a.net_w[e] : 1.0f;
    if (deg <= a.clique_max) {
        int64_t q = q_clique(w, deg);
        int node[kNetUnroll];
        const int c = clique_nodes(a.pin_x, lo, hi, v, node);
        if (!c) return;
        int64_t k = rp[v] + slot[p];
        if (deg <= kNetUnroll) {
#pragma unroll
            for (int u = 0; u < kNetUnroll; ++u)
                if (lo + u < hi && node[u] != v) {
                    raw[k] = raw_ent(node[u], q);
                    ++k;
                }
        } else {
            for (int b = lo; b < hi; ++b) {
                int u = a.pin_x[b];
                if (u == v) continue;
                raw[k] = raw_ent(u, q);
                ++k;
            }
        }
    } else {
        int64_t q = q_star(w, deg);
        int z = a.first_star + a.star_rank[e];
        int64_t k = rp[v] + slot[p];
        raw[k] = raw_ent(z, q);
        int64_t kz = rp[z] + (p - lo);
        raw[kz] = raw_ent(v, q);
    }
}

// Row classes by entry count: 0 (<= 1), 1 (<= 8), 2 (<= 16), 3 (<= 32),
// 4 (<= 64), 5 (longer); classes 1-4 are sorted by 8, 16, 32 and 64 lanes
// per row.
constexpr int kSortClasses = 6;
__device__ __forceinline__ int row_class(int c) {
    return c <= 1 ? 0 : (c <= 8 ? 1 : (c <= 16 ? 2 : (c <= 32 ? 3 : (c <= 64 ? 4 : 5))));
}

__global__ void k_class_keys(const int32_t* __restrict__ cnt, int32_t n, int32_t* __restrict__ key) {
    int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r < n) key[r] = row_class(cnt[r]);
}

// Rows with at most one entry: copy through.
__global__ void k_sort_trivial(const int32_t* __restrict__ rows, int32_t nrows, const int32_t* __restrict__ cnt,
                               const int64_t* __restrict__ rp, const RawEnt* __restrict__ raw,
                               int32_t* __restrict__ scol, int64_t* __restrict__ sq,
                               int32_t* __restrict__ ucnt, int64_t* __restrict__ qdeg) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    int r = rows[i];
    int c = cnt[r];
    ucnt[r] = c;
    int64_t q = 0;
    if (c == 1) {
        const RawEnt e = raw[rp[r]];
        scol[rp[r]] = e.col;
        sq[rp[r]] = e.q;
        q = e.q;
    }
    qdeg[r] = q;
}

// G lanes per row (G = 8, 16, 32 or 64): bitonic sort by column across the lanes,
// then merge equal columns by exact integer sums.  Narrow: the column ids
// leave room for a lane index beside them in 31 bits.
template <int G, bool Narrow>
__global__ void __launch_bounds__(kBT) k_sort_group(const int32_t* __restrict__ rows, int32_t nrows,
                                                    const int32_t* __restrict__ cnt, const int64_t* __restrict__ rp,
                                                    const RawEnt* __restrict__ raw,
                                                    int32_t* __restrict__ scol, int64_t* __restrict__ sq,
                                                    int32_t* __restrict__ ucnt, int64_t* __restrict__ qdeg) {
    int64_t gid = (static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x) / G;
    int l = threadIdx.x & (G - 1);
    int lane = lane_id();
    int gbase = lane - l;      // first lane of this group inside the wave
    bool valid_row = gid < nrows;
    int r = valid_row ? rows[gid] : 0;
    int len = valid_row ? cnt[r] : 0;
    int64_t base = valid_row ? rp[r] : 0;
    int key = 0x7fffffff;
    int64_t q = 0;
    if (l < len) {
        const RawEnt e = raw[base + l];
        key = e.col;
        q = e.q;
    }
    if constexpr (Narrow) {
        // one 32-bit key per lane, (column, lane) packed: unique, so the
        // network moves the key alone and each lane then fetches the weight
        // of the entry it ended up with
        constexpr int LB = G == 8 ? 3 : G == 16 ? 4 : G == 32 ? 5 : 6;
        int ck = l < len ? ((key << LB) | l) : 0x7fffffff;
#pragma unroll
        for (int k = 2; k <= G; k <<= 1) {
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                const int pk = __shfl_xor(ck, j);
                const bool up = (l & k) == 0;
                const bool lower = (l & j) == 0;
                const bool take = lower ? (up ? (pk < ck) : (pk > ck)) : (up ? (pk > ck) : (pk < ck));
                ck = take ? pk : ck;
            }
        }
        q = __shfl(q, gbase + (ck & (G - 1)));
        key = l < len ? (ck >> LB) : 0x7fffffff;
    } else {
#pragma unroll
        for (int k = 2; k <= G; k <<= 1) {
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                int pk = __shfl_xor(key, j);
                int64_t pq = __shfl_xor(q, j);
                bool up = (l & k) == 0;
                bool lower = (l & j) == 0;
                bool take = lower ? (up ? (pk < key) : (pk > key)) : (up ? (pk > key) : (pk < key));
                if (take) {
                    key = pk;
                    q = pq;
                }
            }
        }
    }
    int prev = __shfl(key, gbase + (l > 0 ? l - 1 : 0));
    int next = __shfl(key, gbase + (l + 1 < G ? l + 1 : l));
    bool head = (l < len) && (l == 0 || prev != key);
    bool tail = (l < len) && (l + 1 == len || next != key);
    // run sums from exact int64 prefix sums: sum = pre[l] - pre[start - 1]
    int64_t pre = q;
    int start = head ? l : 0;
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
        int64_t pu = __shfl(pre, gbase + (l >= d ? l - d : l));
        int su = __shfl(start, gbase + (l >= d ? l - d : l));
        if (l >= d) {
            pre += pu;
            start = su > start ? su : start;
        }
    }
    int64_t before = __shfl(pre, gbase + (start > 0 ? start - 1 : 0));
    int64_t sum = pre - (start > 0 ? before : 0);
    uint64_t hm = __ballot(head);
    uint64_t gm = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << gbase);
    uint64_t below_start = (gbase + start) ? (~0ull >> (kWave - (gbase + start))) : 0ull;
    int idx = __popcll(hm & gm & below_start);
    if (tail) {
        scol[base + idx] = key;
        sq[base + idx] = sum;
    }
    if (valid_row && l == 0) ucnt[r] = __popcll(hm & gm);
    if (valid_row && l == G - 1) qdeg[r] = pre;      // the inclusive scan's last lane: the row's weight sum
}

// One workgroup of kLongBT threads per long row (star rows reach 10^4
// entries, so the rows' sorts are spread over many lanes): bitonic sort of
// (column, slot) keys --
// in LDS when the padded row fits `lds_keys` (dynamic shared memory),
// otherwise in the row's own segment of `tkey` (global memory) -- with
// positions past the row end acting as +infinity, then an ordered merge of
// equal columns.
constexpr int kLongBT = 1024;

// Merge sort of a long row's keys (unique 64-bit) by one workgroup, for rows
// of at most kLongBT * kRunMax keys: thread t sorts the E keys from t E on
// in registers (odd-even transposition, fixed indices), then log2(kLongBT)
// merge rounds double the sorted runs.  In a round each thread finds where
// its E outputs start on the merge path of its pair of runs (binary
// search), merges them into registers, and after a barrier writes them back
// in place.  Slots past n hold ~0 and sort last.  O(n log n) LDS traffic,
// against O(n log^2 n) for the bitonic network used for longer rows.
constexpr int kRunMax = 16;

__device__ void block_merge_sort(const RawEnt* __restrict__ raw, int64_t base, int n, int E, uint64_t* key) {
    const int t = threadIdx.x;
    uint64_t v[kRunMax];
#pragma unroll
    for (int u = 0; u < kRunMax; ++u) {
        const int k = t * E + u;
        const bool ok = u < E && k < n;
        const int32_t c = raw[base + (ok ? k : 0)].col;          // every load in flight at once
        v[u] = ok ? (static_cast<uint64_t>(static_cast<uint32_t>(c)) << 32) | static_cast<uint32_t>(k) : ~0ull;
    }
#pragma unroll
    for (int rnd = 0; rnd < kRunMax; ++rnd) {
#pragma unroll
        for (int u = rnd & 1; u + 1 < kRunMax; u += 2) {
            const uint64_t x = v[u], y = v[u + 1];
            v[u] = y < x ? y : x;
            v[u + 1] = y < x ? x : y;
        }
    }
#pragma unroll
    for (int u = 0; u < kRunMax; ++u)
        if (u < E) key[t * E + u] = v[u];
    __syncthreads();
    const int total = kLongBT * E;
    for (int w = E; w < total; w <<= 1) {
        const int d0 = t * E;
        const int s = d0 / (2 * w) * (2 * w);
        const uint64_t* A = key + s;
        const uint64_t* B = key + s + w;
        const int d = d0 - s;
        int lo = d > w ? d - w : 0, hi = d < w ? d : w;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (A[mid] <= B[d - mid - 1]) lo = mid + 1;
            else hi = mid;
        }
        int i = lo, j = d - lo;
#pragma unroll
        for (int u = 0; u < kRunMax; ++u) {
            if (u < E) {
                const uint64_t a = i < w ? A[i] : ~0ull, b = j < w ? B[j] : ~0ull;
                const bool ta = j >= w || (i < w && a <= b);
                v[u] = ta ? a : b;
                i += ta ? 1 : 0;
                j += ta ? 0 : 1;
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kRunMax; ++u)
            if (u < E) key[t * E + u] = v[u];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kLongBT) k_sort_long(const int32_t* __restrict__ rows, const int32_t* __restrict__ cnt,
                                                   const int64_t* __restrict__ rp, const RawEnt* __restrict__ raw,
                                                   uint64_t* __restrict__ tkey,
                                                   int32_t* __restrict__ scol, int64_t* __restrict__ sq,
                                                   int32_t* __restrict__ ucnt, int64_t* __restrict__ qdeg,
                                                   int lds_keys) {
    extern __shared__ uint64_t lkey[];
    __shared__ int red[kLongBT / kWave];
    __shared__ int carry;
    __shared__ unsigned long long qtot;      // the row's weight sum (exact: integer adds)
    int r = rows[blockIdx.x];
    int n = cnt[r];
    int64_t base = rp[r];
    const int E = (n + kLongBT - 1) / kLongBT;
    const bool merge = E <= kRunMax && kLongBT * E <= lds_keys;      // block-uniform
    int P = 1;
    while (P < n) P <<= 1;
    uint64_t* key = merge || P <= lds_keys ? lkey : tkey + base;
    if (merge) {
        block_merge_sort(raw, base, n, E, key);
        P = 0;                                                     // skips the network below
    } else {
        for (int k = threadIdx.x; k < n; k += kLongBT)
            key[k] = (static_cast<uint64_t>(static_cast<uint32_t>(raw[base + k].col)) << 32) | static_cast<uint32_t>(k);
        __threadfence_block();
        __syncthreads();
    }
    for (int size = 2; size <= P; size <<= 1) {
        int half = size >> 1;
        // first comparator layer of a merge: mirror pairs
        for (int i = threadIdx.x; i < P / 2; i += kLongBT) {
            int blk = i / half, off = i % half;
            int a = blk * size + off;
            int b = blk * size + size - 1 - off;
            if (b < n) {
                uint64_t x = key[a], y = key[b];
                if (y < x) { key[a] = y; key[b] = x; }
            }
        }
        __threadfence_block();
        __syncthreads();
        for (int h = half >> 1; h > 0; h >>= 1) {
            for (int i = threadIdx.x; i < P / 2; i += kLongBT) {
                int a = (i / h) * 2 * h + (i % h);
                int b = a + h;
                if (b < n) {
                    uint64_t x = key[a], y = key[b];
                    if (y < x) { key[a] = y; key[b] = x; }
                }
            }
            __threadfence_block();
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        carry = 0;
        qtot = 0;
    }
    __syncthreads();
    for (int t0 = 0; t0 < n; t0 += kLongBT) {
        int k = t0 + threadIdx.x;
        uint32_t col = 0;
        bool head = false;
        if (k < n) {
            col = static_cast<uint32_t>(key[k] >> 32);
            head = (k == 0) || (static_cast<uint32_t>(key[k - 1] >> 32) != col);
        }
        int tot;
        int idx = block_rank<kLongBT>(head, red, &tot);
        if (head) {
            int64_t s = 0;
            for (int m = k; m < n && static_cast<uint32_t>(key[m] >> 32) == col; ++m)
                s += raw[base + static_cast<uint32_t>(key[m] & 0xffffffffu)].q;
            scol[base + carry + idx] = static_cast<int32_t>(col);
            sq[base + carry + idx] = s;
            atomicAdd(&qtot, static_cast<unsigned long long>(s));
        }
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ucnt[r] = carry;
        qdeg[r] = static_cast<int64_t>(qtot);
    }
}

__global__ void k_base_weight(int32_t n_inst, const int32_t* __restrict__ net_len, const int64_t* __restrict__ qdeg,
                              double* __restrict__ bw) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_inst) return;
    int nnz = net_len[i];
    int64_t q = qdeg[i];
    bw[i] = (nnz > 0 && q != 0) ? (static_cast<double>(q) * 0x1p-32) / static_cast<double>(nnz) : 0.0;
}

// Keys of a long row that one workgroup sorts in LDS: the largest power of
// two whose keys fit the per-workgroup shared memory with 1 KiB to spare.
int sort_lds_keys(int device) {
    static int cached[64] = {0};
    if (device >= 0 && device < 64 && cached[device]) return cached[device];
    hipDeviceProp_t prop;
    AHR_HIP(hipGetDeviceProperties(&prop, device));
    size_t avail = prop.sharedMemPerBlock > 1024 ? prop.sharedMemPerBlock - 1024 : 0;
    int k = 1;
    while (static_cast<size_t>(k) * 2 * sizeof(uint64_t) <= avail && k < (1 << 16)) k <<= 1;
    if (device >= 0 && device < 64) cached[device] = k;
    return k;
}

}  // namespace

void build_netlist(Graph& g, hipStream_t s) {
    ProfScope ps(kStageBuild, s);
    const ahr_netlist& nl = g.nl;
    const int32_t n_pins = nl.n_pins, n_nets = nl.n_nets, n_inst = nl.n_inst;
    const ahr_hint_params& hp = g.hp;

    // validate the device arrays
    g.counter.ensure(8, s);
    fill_i32(g.counter.p, 8, 0, s);
    int64_t nv = (n_pins > n_nets + 1) ? n_pins : static_cast<int64_t>(n_nets) + 1;
    hipLaunchKernelGGL(k_validate, dim3(grid_for(nv, kBT)), dim3(kBT), 0, s, nl.net_ptr, n_nets, nl.pin_node, n_pins,
                       n_inst, g.counter.p);
    AHR_LAUNCHED("k_validate");
    // The verdict is read together with the counts below: the kernels in
    // between index only with clamped pin nodes, so an invalid netlist reads
    // nothing out of bounds before it is rejected.

    // flags of macro pins, star nets, big nets, macros; their ranks; one read of the four counts
    DevBuf<int32_t> is_mp, mp_rank, is_star, star_rank, is_big, big_rank, is_mac, mac_rank, is_bs, bs_rank;
    is_mp.ensure(static_cast<size_t>(n_pins) + 1, s);
    is_star.ensure(static_cast<size_t>(n_nets) + 1, s);
    is_big.ensure(static_cast<size_t>(n_nets) + 1, s);
    is_bs.ensure(static_cast<size_t>(n_nets) + 1, s);
    is_mac.ensure(static_cast<size_t>(n_inst) + 1, s);
    if (n_pins)
        hipLaunchKernelGGL(k_mark_mpin, dim3(grid_for(n_pins, kBT)), dim3(kBT), 0, s, nl.pin_node, nl.node_flags,
                           n_pins, n_inst, (hp.flags & AHR_EXPAND_MACRO_PINS) ? 1 : 0, is_mp.p);
    AHR_LAUNCHED("k_mark_mpin");
    if (n_nets)
        hipLaunchKernelGGL(k_mark_star, dim3(grid_for(n_nets, kBT)), dim3(kBT), 0, s, nl.net_ptr, n_nets,
                           hp.clique_max, is_star.p, is_big.p, is_bs.p);
    AHR_LAUNCHED("k_mark_star");
    hipLaunchKernelGGL(k_mark_macro, dim3(grid_for(n_inst, kBT)), dim3(kBT), 0, s, nl.node_flags, n_inst, is_mac.p,
                       g.counter.p + 1);
    AHR_LAUNCHED("k_mark_macro");
    mp_rank.ensure(static_cast<size_t>(n_pins) + 1, s);
    star_rank.ensure(static_cast<size_t>(n_nets) + 1, s);
    big_rank.ensure(static_cast<size_t>(n_nets) + 1, s);
    bs_rank.ensure(static_cast<size_t>(n_nets) + 1, s);
    mac_rank.ensure(static_cast<size_t>(n_inst) + 1, s);
    g.scan_tmp.ensure(scan_tmp_elems(std::max<int64_t>(std::max<int64_t>(n_pins, n_nets), n_inst)), s);
    scan_i32_to_i32(is_mp.p, mp_rank.p, n_pins, g.scan_tmp.p, s);
    scan_i32_to_i32(is_star.p, star_rank.p, n_nets, g.scan_tmp.p, s);
    scan_i32_to_i32(is_big.p, big_rank.p, n_nets, g.scan_tmp.p, s);
    scan_i32_to_i32(is_mac.p, mac_rank.p, n_inst, g.scan_tmp.p, s);
    scan_i32_to_i32(is_bs.p, bs_rank.p, n_nets, g.scan_tmp.p, s);
    int32_t cnt5[7];
    read_scalars({mp_rank.p + n_pins, star_rank.p + n_nets, big_rank.p + n_nets, mac_rank.p + n_inst,
                  bs_rank.p + n_nets, g.counter.p, g.counter.p + 1},
                 cnt5, s);
    if (const int32_t bad = cnt5[5]) {
        static const char* why[] = {"", "pin_node out of [0, n_inst)", "net_ptr[0] != 0",
                                    "net_ptr[n_nets] != n_pins", "net_ptr decreasing"};
        throw Error{AHR_EINVAL, std::string("invalid netlist: ") + why[bad]};
    }
    g.n_mpin = cnt5[0];
    g.n_star = cnt5[1];
    g.n_big_nets = cnt5[2];
    g.n_macro = cnt5[3];
    g.n_big_stars = cnt5[4];
    g.n_movable_macro = cnt5[6];
    if ((hp.flags & AHR_MACRO_HINTS) && g.n_macro > 16384)
        throw Error{AHR_EUNSUPPORTED, "macro hints support at most 16384 macros"};
    g.star_net.ensure(static_cast<size_t>(g.n_star) + 1, s);
    g.big_nets.ensure(static_cast<size_t>(g.n_big_nets) + 1, s);
    g.macro_ids.ensure(static_cast<size_t>(g.n_macro) + 1, s);
    list_rows(is_star.p, star_rank.p, n_nets, g.star_net.p, s);
    list_rows(is_big.p, big_rank.p, n_nets, g.big_nets.p, s);
    list_rows(is_mac.p, mac_rank.p, n_inst, g.macro_ids.p, s);
    // stars averaged by a whole workgroup
    g.big_stars.ensure(static_cast<size_t>(g.n_big_stars) + 1, s);
    if (n_nets)
        hipLaunchKernelGGL(k_list_big_stars, dim3(grid_for(n_nets, kBT)), dim3(kBT), 0, s, is_bs.p, bs_rank.p,
                           star_rank.p, n_nets, g.big_stars.p);
    AHR_LAUNCHED("k_list_big_stars");
    is_bs.release(s);
    bs_rank.release(s);
    g.pin_node_x.ensure(static_cast<size_t>(n_pins) + 1, s);
    g.mpin_owner.ensure(static_cast<size_t>(g.n_mpin) + 1, s);
    g.mpin_pin.ensure(static_cast<size_t>(g.n_mpin) + 1, s);
    if (n_pins)
        hipLaunchKernelGGL(k_pin_nodes, dim3(grid_for(n_pins, kBT)), dim3(kBT), 0, s, nl.pin_node, is_mp.p, mp_rank.p,
                           n_pins, n_inst, g.pin_node_x.p, g.mpin_owner.p, g.mpin_pin.p);
    AHR_LAUNCHED("k_pin_nodes");
    is_mp.release(s);
    mp_rank.release(s);
    is_big.release(s);
    big_rank.release(s);
    is_mac.release(s);
    mac_rank.release(s);

    // node ranges
    int64_t first_mpin = n_inst;
    int64_t first_star = first_mpin + g.n_mpin;
    int64_t first_mvirt = first_star + g.n_star;
    int64_t n_mv = (hp.flags & AHR_MACRO_HINTS) ? g.n_macro : 0;
    int64_t first_bvirt = first_mvirt + n_mv;
    int64_t n_bins = (hp.flags & AHR_BIN_HINTS) ? static_cast<int64_t>(hp.nbx) * hp.nby : 0;
    int64_t n_tot = first_bvirt + n_bins;
    if (n_tot >= INT32_MAX) throw Error{AHR_EUNSUPPORTED, "graph has 2^31 or more nodes"};
    g.first_mpin = static_cast<int32_t>(first_mpin);
    g.first_star = static_cast<int32_t>(first_star);
    g.first_mvirt = static_cast<int32_t>(first_mvirt);
    g.first_bvirt = static_cast<int32_t>(first_bvirt);
    g.n_bins = static_cast<int32_t>(n_bins);
    g.n_tot = static_cast<int32_t>(n_tot);
    g.n_inst = n_inst;
    const int32_t N = g.n_tot;

    // net of every pin, then entry counts per row (parallel edges counted)
    DevBuf<int32_t> pin_net;
    pin_net.ensure(static_cast<size_t>(n_pins) + 1, s);
    if (n_nets)
        hipLaunchKernelGGL(k_pin_net, dim3(grid_for(n_nets, kBT)), dim3(kBT), 0, s, nl.net_ptr, n_nets, pin_net.p);
    AHR_LAUNCHED("k_pin_net");
    if (g.n_big_nets) {
        hipLaunchKernelGGL(k_pin_net_big, dim3(g.n_big_nets), dim3(kBT), 0, s, g.big_nets.p, nl.net_ptr, pin_net.p);
        AHR_LAUNCHED("k_pin_net_big");
    }
    NetArgs a{nl.net_ptr, pin_net.p, g.pin_node_x.p, nl.net_w, star_rank.p, n_nets, n_pins, hp.clique_max,
              g.first_star};
    DevBuf<int32_t> cnt, slot;
    cnt.ensure(static_cast<size_t>(N) + 1, s);
    fill_i32(cnt.p, N + 1, 0, s);
    slot.ensure(static_cast<size_t>(n_pins) + 1, s);
    if (n_pins)
        hipLaunchKernelGGL(k_row_counts, dim3(grid_for(n_pins, kBT)), dim3(kBT), 0, s, a, cnt.p, slot.p);
    AHR_LAUNCHED("k_row_counts");
    // the rows stay where the raw entries put them: net_off[r] is row r's
    // first slot, net_len[r] its merged entry count (set by the sorts)
    DevBuf<int64_t>& rp = g.net_off;
    rp.ensure(static_cast<size_t>(N) + 1, s);
    g.scan_tmp.ensure(scan_tmp_elems(N), s);
    scan_i32_to_i64(cnt.p, rp.p, N, g.scan_tmp.p, s);
    // rows grouped by length class (ascending rows within a class), read
    // with the raw entry total
    constexpr int K = kSortClasses;
    DevBuf<int32_t> ckey, lists, cstart;
    ckey.ensure(static_cast<size_t>(N) + 1, s);
    hipLaunchKernelGGL(k_class_keys, dim3(grid_for(N, kBT)), dim3(kBT), 0, s, cnt.p, N, ckey.p);
    AHR_LAUNCHED("k_class_keys");
    bucket_sort(g, ckey.p, N, K, lists, cstart, s, false);
    ckey.release(s);
    int64_t w[K + 2];
    read_words({{rp.p + N, 1}, {cstart.p, 0}, {cstart.p + 1, 0}, {cstart.p + 2, 0}, {cstart.p + 3, 0},
                {cstart.p + 4, 0}, {cstart.p + 5, 0}, {cstart.p + 6, 0}},
               w, s);
    static_assert(K == 6, "class starts read above");
    const int64_t nnz_dup = w[0];
    if (nnz_dup >= INT32_MAX) throw Error{AHR_EUNSUPPORTED, "netlist expands to 2^31 or more graph entries"};
    int32_t ncls[K];
    const int32_t* cls[K];
    for (int k = 0; k < K; ++k) {
        ncls[k] = static_cast<int32_t>(w[2 + k] - w[1 + k]);
        cls[k] = lists.p + w[1 + k];
    }

    DevBuf<int32_t>& scol = g.net_col;
    DevBuf<int32_t>& ucnt = g.net_len;
    DevBuf<RawEnt> raw;
    DevBuf<int64_t>& sq = g.net_q;
    raw.ensure(static_cast<size_t>(nnz_dup) + 1, s);
    if (n_pins)
        hipLaunchKernelGGL(k_scatter, dim3(grid_for(n_pins, kBT)), dim3(kBT), 0, s, a, rp.p, slot.p, raw.p);
    AHR_LAUNCHED("k_scatter");
    slot.release(s);
    pin_net.release(s);
    is_star.release(s);
    star_rank.release(s);

    // per-row sort + merge by length class
    scol.ensure(static_cast<size_t>(nnz_dup) + 1, s);
    sq.ensure(static_cast<size_t>(nnz_dup) + 1, s);
    ucnt.ensure(static_cast<size_t>(N) + 1, s);
    fill_i32(ucnt.p, N + 1, 0, s);
    g.qdeg.ensure(static_cast<size_t>(N) + 1, s);
    if (ncls[0])
        hipLaunchKernelGGL(k_sort_trivial, dim3(grid_for(ncls[0], kBT)), dim3(kBT), 0, s, cls[0], ncls[0], cnt.p,
                           rp.p, raw.p, scol.p, sq.p, ucnt.p, g.qdeg.p);
    AHR_LAUNCHED("k_sort_trivial");
    // rows of up to 64 entries sort (column, lane) pairs packed in 32 bits
    const bool narrow = N < (1 << 25);
    if (ncls[1])
        hipLaunchKernelGGL((narrow ? k_sort_group<8, true> : k_sort_group<8, false>),
                           dim3(grid_for(static_cast<int64_t>(ncls[1]) * 8, kBT)), dim3(kBT), 0, s,
                           cls[1], ncls[1], cnt.p, rp.p, raw.p, scol.p, sq.p, ucnt.p, g.qdeg.p);
    AHR_LAUNCHED("k_sort_group8");
    if (ncls[2])
        hipLaunchKernelGGL((narrow ? k_sort_group<16, true> : k_sort_group<16, false>),
                           dim3(grid_for(static_cast<int64_t>(ncls[2]) * 16, kBT)), dim3(kBT), 0, s,
                           cls[2], ncls[2], cnt.p, rp.p, raw.p, scol.p, sq.p, ucnt.p, g.qdeg.p);
    AHR_LAUNCHED("k_sort_group16");
    if (ncls[3])
        hipLaunchKernelGGL((narrow ? k_sort_group<32, true> : k_sort_group<32, false>),
                           dim3(grid_for(static_cast<int64_t>(ncls[3]) * 32, kBT)), dim3(kBT), 0, s,
                           cls[3], ncls[3], cnt.p, rp.p, raw.p, scol.p, sq.p, ucnt.p, g.qdeg.p);
    AHR_LAUNCHED("k_sort_group32");
    if (ncls[4])
        hipLaunchKernelGGL((narrow ? k_sort_group<64, true> : k_sort_group<64, false>),
                           dim3(grid_for(static_cast<int64_t>(ncls[4]) * 64, kBT)), dim3(kBT), 0, s,
                           cls[4], ncls[4], cnt.p, rp.p, raw.p, scol.p, sq.p, ucnt.p, g.qdeg.p);
    AHR_LAUNCHED("k_sort_group64");
    if (ncls[5]) {
        DevBuf<uint64_t> tkey;
        tkey.ensure(static_cast<size_t>(nnz_dup) + 1, s);
        const int lds_keys = sort_lds_keys(g.device);
        hipLaunchKernelGGL(k_sort_long, dim3(ncls[5]), dim3(kLongBT), static_cast<size_t>(lds_keys) * sizeof(uint64_t), s,
                           cls[5], cnt.p, rp.p, raw.p, tkey.p, scol.p, sq.p, ucnt.p, g.qdeg.p, lds_keys);
        AHR_LAUNCHED("k_sort_long");
        tkey.release(s);
    }
    raw.release(s);

    // The merged rows stay in place (no compaction): slots past a row's
    // merged count are unused.  The arrays hold the raw count; the exact
    // entry count is read later with other sizes.
    g.nnz_net = -1;
    g.nnz_cap = static_cast<int32_t>(nnz_dup);
    lists.release(s);
    cstart.release(s);
    g.base_w.ensure(static_cast<size_t>(n_inst) + 1, s);
    hipLaunchKernelGGL(k_base_weight, dim3(grid_for(n_inst, kBT)), dim3(kBT), 0, s, n_inst, g.net_len.p, g.qdeg.p,
                       g.base_w.p);
    AHR_LAUNCHED("k_base_weight");
    cnt.release(s);
}

}  // namespace ahr
