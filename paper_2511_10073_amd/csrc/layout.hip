// Execution layout of the filter.  Instance ids arrive in netlist order,
// which carries no locality, so neighbour gathers of the SpMM hop would each
// touch a different cache line.  The filter therefore streams rows in an
// execution order: instances sorted by a stable sort on the Hilbert-curve
// index of their position on a 1024 x 1024 grid over the die, columns
// renumbered to match.  The macro pin nodes and the star nodes stay in their
// own id ranges but are ordered the same way inside them (a macro pin by its
// pin position, a star by the position of its net's first pin), so that the
// rows gathering a run of them, and their own rows, touch few cache lines;
// the virtual nodes keep their canonical ids.  Consecutive rows are then spatial neighbours, so the
// rows of one workgroup gather from few, shared cache lines, and every
// aligned power-of-two block of the grid (a bin of a 2^k x 2^k bin grid) is
// one contiguous range of rows.  Inside each aligned window of 64 rows (the
// rows of one workgroup of the hop) the rows are then ordered by netlist
// row length, so the rows that share a wave need about the same number of
// entry batches and the window stays one spatial neighbourhood.  The
// netlist rows are copied into that order, the entries of each short row
// sorted by their renumbered column (so a row's gathers also walk the
// layout in order; the summation order is fixed by the inputs and the first
// placement); the hint rows are built in it directly.  The canonical netlist
// CSR stays for export; the order is set once per graph from the first
// placement seen.
//
// A placement whose positions say little about the netlist (uniformly
// drawn ones, or a low-order smoothing of them) gives a Hilbert order with
// no locality.  On request (AHR_LAYOUT_NETLIST) the instances take a
// netlist order instead: Cuthill-McKee levels over the instance-to-instance
// netlist edges (star and macro pin nodes left out, since a big net reaches
// across the die), a node's rank following its lowest-ranked parent,
// siblings in id order; macro pin and star rows follow the lowest rank among
// their instance neighbours.  With AHR_LAYOUT_AUTO the Hilbert order is kept
// when at least a quarter of a sample of its instance-to-instance entries lie
// within n_inst/64 rows (at least 256) of their row (a random order puts
// about 1/32 of them there), else the netlist order is taken.
#include "ahr_internal.hpp"
#include "device_util.hpp"

namespace ahr {

namespace {

constexpr int kBT = 256;
constexpr int kGridBits = 10;    // 1024 x 1024 layout grid -> 20-bit Hilbert keys
constexpr int kKeyBits = 22;     // the node range (instance, macro pin, star) above them
constexpr int kDigitBits = 11;   // sorted as two stable 11-bit digit passes

// Hilbert-curve index of grid cell (x, y) on the 2^kGridBits square grid:
// at each level the quadrant's position along the curve, then the cell's
// coordinates reflected into that quadrant's orientation.
__device__ __forceinline__ int hilbert_index(int x, int y) {
    int d = 0;
    for (int s = 1 << (kGridBits - 1); s > 0; s >>= 1) {
        const int rx = (x & s) ? 1 : 0, ry = (y & s) ? 1 : 0;
        d += s * s * ((3 * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = s - 1 - x;
                y = s - 1 - y;
            }
            const int t = x;
            x = y;
            y = t;
        }
    }
    return d;
}

struct KeyArgs {
    const float* pos;            // instance positions, ncols per row
    int ncols;
    int32_t n_inst, first_star, first_mvirt;
    const int32_t* mpin_pin;     // pin of each macro pin node
    const int32_t* star_net;     // net of each star node
    const int32_t* net_ptr;
    const int32_t* pin_node;     // instance of each pin
    const int32_t* pin_node_x;   // node of each pin (macro pins expanded)
    const float* pin_off;
    float xl, yl, sx, sy;
};

// Position of pin p: its instance's, plus the pin offset where the pin is
// its own node.
__device__ __forceinline__ float2 pin_pos(const KeyArgs& a, int p) {
    const int v = a.pin_node[p];
    float x = a.pos[static_cast<int64_t>(v) * a.ncols], y = a.pos[static_cast<int64_t>(v) * a.ncols + 1];
    if (a.pin_node_x[p] >= a.n_inst) {
        x += a.pin_off[2 * p];
        y += a.pin_off[2 * p + 1];
    }
    return make_float2(x, y);
}

// Sort key of node i < first_mvirt: its range above the Hilbert index of
// its position.
__global__ void k_layout_keys(KeyArgs a, int32_t* __restrict__ key, int32_t* __restrict__ lo) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.first_mvirt) return;
    float2 q;
    int range;
    if (i < a.n_inst) {
        q = make_float2(a.pos[i * a.ncols], a.pos[i * a.ncols + 1]);
        range = 0;
    } else if (i < a.first_star) {
        q = pin_pos(a, a.mpin_pin[i - a.n_inst]);
        range = 1;
    } else {
        q = pin_pos(a, a.net_ptr[a.star_net[i - a.first_star]]);
        range = 2;
    }
    const int m = (1 << kGridBits) - 1;
    float fx = floorf((q.x - a.xl) * a.sx);
    float fy = floorf((q.y - a.yl) * a.sy);
    int gx = !(fx > 0.f) ? 0 : (fx >= static_cast<float>(m) ? m : static_cast<int>(fx));
    int gy = !(fy > 0.f) ? 0 : (fy >= static_cast<float>(m) ? m : static_cast<int>(fy));
    const int k = (range << (2 * kGridBits)) | hilbert_index(gx, gy);
    key[i] = k;
    lo[i] = k & ((1 << kDigitBits) - 1);
}

// Second digit pass: the high digit of the key of each element of the
// first pass's order.
__global__ void k_high_digit(int32_t n, const int32_t* __restrict__ key, const int32_t* __restrict__ order,
                             int32_t* __restrict__ hi) {
    int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j < n) hi[j] = key[order[j]] >> kDigitBits;
}

__global__ void k_compose(int32_t n, const int32_t* __restrict__ first, const int32_t* __restrict__ second,
                          int32_t* __restrict__ perm) {
    int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r < n) perm[r] = first[second[r]];
}

// Stable sort of each aligned window of kLenWindow positions of `in` by the
// netlist row length of its instance (one wave per window): the rank of an
// element is the number of elements of its window with a smaller length, or
// the same length and an earlier position.
constexpr int kLenWindow = 64;

__global__ void __launch_bounds__(kLenWindow) k_window_sort(int32_t n, const int32_t* __restrict__ in,
                                                            const int32_t* __restrict__ net_len,
                                                            int32_t* __restrict__ out) {
    __shared__ int32_t wlen[kLenWindow];
    const int t = threadIdx.x;
    const int64_t j = static_cast<int64_t>(blockIdx.x) * kLenWindow + t;
    int32_t id = 0, len = INT32_MAX;                 // positions past n sort last and are not written
    if (j < n) {
        id = in[j];
        len = net_len[id];
    }
    wlen[t] = len;
    __syncthreads();
    int rank = 0;
    for (int u = 0; u < kLenWindow; ++u) {
        const int32_t o = wlen[u];
        rank += (o < len || (o == len && u < t)) ? 1 : 0;
    }
    if (j < n) out[static_cast<int64_t>(blockIdx.x) * kLenWindow + rank] = id;
}

// Both directions over all n_tot rows: the virtual rows (from n_perm on)
// map to themselves.
__global__ void k_iperm(int32_t* __restrict__ perm, int32_t n_perm, int32_t n_tot, int32_t* __restrict__ iperm) {
    int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r < n_perm) {
        iperm[perm[r]] = static_cast<int32_t>(r);
    } else if (r < n_tot) {
        perm[r] = static_cast<int32_t>(r);
        iperm[r] = static_cast<int32_t>(r);
    }
}


// Per execution row, from its node: the netlist row length, the row weight
// sum, and for the macro pin and star rows what the expansion reads (a
// macro pin's owner instance and pin offset, a star's net).
struct ExecRowArgs {
    int32_t n_tot, n_inst, first_star, first_mvirt;
    const int32_t* perm;
    const int32_t* net_len;
    const int64_t* qdeg;
    const int32_t* mpin_pin;
    const int32_t* pin_node;
    const float* pin_off;
    const int32_t* star_net;
    int32_t* len;
    int64_t* xqdeg;
    int4* xmpin;
    int32_t* xstar_net;
};

__global__ void k_exec_rows(ExecRowArgs a) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= a.n_tot) return;
    const int v = a.perm[r];
    a.len[r] = a.net_len[v];
    a.xqdeg[r] = a.qdeg[v];
    if (r >= a.n_inst && r < a.first_star) {
        const int p = a.mpin_pin[v - a.n_inst];
        a.xmpin[r - a.n_inst] =
            make_int4(a.pin_node[p], __float_as_int(a.pin_off[2 * p]), __float_as_int(a.pin_off[2 * p + 1]), 0);
    } else if (r >= a.first_star && r < a.first_mvirt) {
        a.xstar_net[r - a.first_star] = a.star_net[v - a.first_star];
    }
}

// Execution-order netlist rows: each row copies its canonical row's
// entries with columns renumbered and weights as float32.  Rows of at most
// kShortRow entries are put in ascending order of the renumbered column, so
// that the lanes of a row gather neighbouring nodes in turn (a row's columns
// are distinct, so an entry's place is the count of smaller ones); G lanes
// per such row.  Longer rows keep their canonical entry order and have one
// workgroup each (k_exec_net_long).
constexpr int kShortRow = 64;

__device__ __forceinline__ int2 exec_entry(int32_t c, int64_t q, const int32_t* iperm) {
    return make_int2(iperm[c], f_bits(static_cast<float>(static_cast<double>(q) * 0x1p-32)));
}

__global__ void __launch_bounds__(kBT) k_exec_net(int32_t n_tot, const int32_t* __restrict__ perm,
                                                  const int32_t* __restrict__ iperm, const int64_t* __restrict__ off,
                                                  const int32_t* __restrict__ col, const int64_t* __restrict__ q,
                                                  const int32_t* __restrict__ xrp, int2* __restrict__ xent) {
    constexpr int G = 8, U = kShortRow / G;
    __shared__ int32_t cols[kBT / G][kShortRow];
    const int64_t r = (static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x) / G;
    const int l = threadIdx.x & (G - 1);
    int32_t* mine = cols[threadIdx.x / G];
    int d = 0, len = 0;
    if (r < n_tot) {
        d = xrp[r];
        len = xrp[r + 1] - d;
        if (len > kShortRow) len = 0;                      // group-uniform: k_exec_net_long
    }
    // No branch around any global load, so that all of a lane's loads are in
    // flight together: indexes are clamped to the row's last entry.
    int32_t m[U];
    int2 e[U];
    if (len > 0) {
        const int64_t a = off[perm[r]];
        int32_t c[U];
        int64_t w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = l + u * G < len ? l + u * G : len - 1;
            c[u] = col[a + k];
            w[u] = q[a + k];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) m[u] = iperm[c[u]];
        // slots past the row's end hold repeats; the counts read below len only
#pragma unroll
        for (int u = 0; u < U; ++u) {
            mine[l + u * G] = m[u];
            e[u] = make_int2(m[u], f_bits(static_cast<float>(static_cast<double>(w[u]) * 0x1p-32)));
        }
    }
    __syncthreads();
    if (len == 0) return;
    // (every load is consumed by now, so a guarded store waits for nothing)
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (l + u * G < len) {
            int rank = 0;
            for (int j = 0; j < len; ++j) rank += mine[j] < m[u] ? 1 : 0;
            xent[static_cast<int64_t>(d) + rank] = e[u];
        }
    }
}

// One workgroup per longer row; the workgroups stride over the list of
// long rows, whose length they read from the device (*n_long).
constexpr int kLongRowGrid = 512;

__global__ void __launch_bounds__(kBT) k_exec_net_long(const int32_t* __restrict__ rows,
                                                       const int32_t* __restrict__ n_long,
                                                       const int32_t* __restrict__ perm,
                                                       const int32_t* __restrict__ iperm,
                                                       const int64_t* __restrict__ off, const int32_t* __restrict__ col,
                                                       const int64_t* __restrict__ q, const int32_t* __restrict__ xrp,
                                                       int2* __restrict__ xent) {
    const int nl = *n_long;
    for (int li = blockIdx.x; li < nl; li += gridDim.x) {
        const int r = rows[li];
        const int d = xrp[r], len = xrp[r + 1] - d;
        const int64_t a = off[perm[r]];
        for (int k = threadIdx.x; k < len; k += kBT) xent[d + k] = exec_entry(col[a + k], q[a + k], iperm);
    }
}

__global__ void k_long_flags(int32_t n_tot, const int32_t* __restrict__ xrp, int32_t* __restrict__ flag) {
    int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r < n_tot) flag[r] = (xrp[r + 1] - xrp[r] > kShortRow) ? 1 : 0;
}


// ---------------------------------------------------------------- netlist order

constexpr int kCmGrid = 1024;       // workgroups of the level kernels (grid-stride over the level)
constexpr int kSample = 64;         // every kSample-th instance row is tested

struct CmArgs {
    int32_t n_inst;
    const int64_t* off;    // canonical netlist rows: off, merged length, columns
    const int32_t* len;
    const int32_t* col;
    unsigned long long* lk;  // [n_inst] BFS level (high word) above the rank of the
                             // lowest-ranked parent; all ones while unvisited
    int32_t* rank;         // [n_inst] position in the order, -1 unplaced
    int32_t* order;        // [n_inst] rank -> instance
    int32_t* cnt;          // [n_inst] children per rank (the current level's ranks)
    const int32_t* scn;    // exclusive scan of cnt ([n_inst] + total)
    int32_t* bnd;          // [0] lo, [1] hi: ranks of the current level; [2] start node
};

__global__ void k_cm_init(CmArgs a) {
    const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v < a.n_inst) {
        a.lk[v] = ~0ull;
        a.rank[v] = -1;
        a.cnt[v] = 0;
    }
    if (v == 0) a.bnd[2] = INT32_MAX;
}

// The start: the lowest instance with an instance neighbour (one atomic per
// wave).
__global__ void __launch_bounds__(kBT) k_cm_start(CmArgs a) {
    const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    int best = INT32_MAX;
    if (v < a.n_inst) {
        const int64_t o = a.off[v];
        const int l = a.len[v];
        for (int k = 0; k < l; ++k)
            if (a.col[o + k] < a.n_inst) {
                best = static_cast<int>(v);
                break;
            }
    }
    best = wave_min(best);
    // (a wave whose candidate cannot lower the current one skips the atomic:
    // the start is nearly always among the first ids)
    if (lane_id() == 0 && best < __hip_atomic_load(&a.bnd[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMin(&a.bnd[2], best);
}

__global__ void k_cm_seed(CmArgs a) {
    int v0 = a.bnd[2];
    if (v0 == INT32_MAX) v0 = 0;            // no instance edges: the order is the id order
    a.lk[v0] = 0ull;
    a.rank[v0] = 0;
    a.order[0] = v0;
    a.bnd[0] = 0;
    a.bnd[1] = 1;
}

// The level kernels give each row of the level kCmLanes lanes, which take
// its entries in turn; the rows of a level are strided over the grid.
constexpr int kCmLanes = 8;

// The packed word of a node of level k + 1 whose lowest-ranked parent is rank i.
__device__ __forceinline__ unsigned long long cm_word(int32_t k, int64_t i) {
    return (static_cast<unsigned long long>(k + 1) << 32) | static_cast<unsigned>(i);
}

__device__ __forceinline__ bool cm_child(const CmArgs& a, int c, int32_t k, int64_t i) {
    return c < a.n_inst && a.lk[c] == cm_word(k, i);
}

// Level k (ranks [lo, hi)): every unvisited instance neighbour joins level
// k + 1 and keeps the lowest rank among its parents, both by one 64-bit
// minimum (an earlier level's word is below every level k + 1 word, an
// unvisited node's above).
__global__ void __launch_bounds__(256) k_cm_expand(CmArgs a, int32_t k) {
    const int lo = a.bnd[0], hi = a.bnd[1];
    const int ln = threadIdx.x & (kCmLanes - 1);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * (blockDim.x / kCmLanes);
    for (int64_t i = lo + (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kCmLanes; i < hi;
         i += stride) {
        const int u = a.order[i];
        const int64_t o = a.off[u];
        const int l = a.len[u];
        const unsigned long long w = cm_word(k, i);
        for (int j = ln; j < l; j += kCmLanes) {
            const int c = a.col[o + j];
            if (c < a.n_inst && a.lk[c] > w) atomicMin(&a.lk[c], w);
        }
    }
}

// Children of each rank of the level: its neighbours whose lowest parent it is.
__global__ void __launch_bounds__(256) k_cm_count(CmArgs a, int32_t k) {
    const int lo = a.bnd[0], hi = a.bnd[1];
    const int ln = threadIdx.x & (kCmLanes - 1);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * (blockDim.x / kCmLanes);
    for (int64_t i = lo + (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kCmLanes; i < hi;
         i += stride) {
        const int u = a.order[i];
        const int64_t o = a.off[u];
        const int l = a.len[u];
        int n = 0;
        for (int j = ln; j < l; j += kCmLanes) n += cm_child(a, a.col[o + j], k, i) ? 1 : 0;
#pragma unroll
        for (int m = kCmLanes / 2; m > 0; m >>= 1) n += __shfl_xor(n, m);   // the row's lanes
        if (ln == 0) a.cnt[i] = n;
    }
}

// Ranks of level k + 1: the children of rank i follow those of the ranks
// before it, each parent's in ascending id (its row is column-sorted; the
// row's lanes place each batch of kCmLanes entries by a ballot).
__global__ void __launch_bounds__(256) k_cm_assign(CmArgs a, int32_t k) {
    const int lo = a.bnd[0], hi = a.bnd[1];
    const int base0 = a.scn[lo];
    const int ln = threadIdx.x & (kCmLanes - 1);
    const int gb = lane_id() & ~(kCmLanes - 1);              // the row's first lane in the wave
    const int64_t stride = static_cast<int64_t>(gridDim.x) * (blockDim.x / kCmLanes);
    for (int64_t i = lo + (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kCmLanes; i < hi;
         i += stride) {
        const int u = a.order[i];
        const int64_t o = a.off[u];
        const int l = a.len[u];
        int r = hi + (a.scn[i] - base0);
        for (int j0 = 0; j0 < l; j0 += kCmLanes) {
            const int j = j0 + ln;
            int c = 0;
            bool f = false;
            if (j < l) {
                c = a.col[o + j];
                f = cm_child(a, c, k, i);
            }
            const unsigned gm = static_cast<unsigned>(__ballot(f) >> gb) & ((1u << kCmLanes) - 1u);
            if (f) {
                const int p = r + __popc(gm & ((1u << ln) - 1u));
                a.rank[c] = p;
                a.order[p] = c;
            }
            r += __popc(gm);
        }
    }
}

// The next level's rank range.
__global__ void k_cm_next(CmArgs a) {
    const int lo = a.bnd[0], hi = a.bnd[1];
    const int nchild = a.scn[hi] - a.scn[lo];
    a.bnd[0] = hi;
    a.bnd[1] = hi + nchild;
}

// Instances the levels never reached (other components, isolated ones):
// after the reached ones, in id order.
__global__ void k_cm_unplaced(int32_t n, const int32_t* __restrict__ rank, int32_t* __restrict__ flag) {
    const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v < n) flag[v] = rank[v] < 0 ? 1 : 0;
}

__global__ void k_cm_append(int32_t n, const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                            const int32_t* __restrict__ bnd, int32_t* __restrict__ rank) {
    const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v < n && flag[v]) rank[v] = bnd[1] + pos[v];
}

// Sort keys of the netlist order (24 bits: range above the rank): an
// instance's own rank, a macro pin's or star's lowest instance-neighbour
// rank (n_inst if none; one wave per such row); low 12 bits to `lo`.
__global__ void k_cm_keys(int32_t n_inst, const int32_t* __restrict__ rank, int32_t* __restrict__ key,
                          int32_t* __restrict__ lo) {
    const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= n_inst) return;
    const int k = rank[v];
    key[v] = k;
    lo[v] = k & 0xfff;
}

__global__ void __launch_bounds__(kBT) k_cm_keys_aux(int32_t n_inst, int32_t np, int32_t first_star,
                                                     const int64_t* __restrict__ off,
                                                     const int32_t* __restrict__ len,
                                                     const int32_t* __restrict__ col,
                                                     const int32_t* __restrict__ rank, int32_t* __restrict__ key,
                                                     int32_t* __restrict__ lo) {
    const int64_t v = n_inst + (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
    if (v >= np) return;                                   // wave-uniform
    const int64_t o = off[v];
    const int l = len[v];
    int r = n_inst;
    for (int j = lane_id(); j < l; j += kWave) {
        const int c = col[o + j];
        if (c < n_inst) r = rank[c] < r ? rank[c] : r;
    }
    r = wave_min(r);
    if (lane_id() == 0) {
        const int k = ((v < first_star ? 1 : 2) << 22) | r;
        key[v] = k;
        lo[v] = k & 0xfff;
    }
}

__global__ void k_hi12(int32_t n, const int32_t* __restrict__ key, const int32_t* __restrict__ order,
                       int32_t* __restrict__ hi) {
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j < n) hi[j] = key[order[j]] >> 12;
}

// Locality of a layout: of a sample of instance rows (every kSample-th
// instance, kNearLanes lanes each), how many instance-to-instance entries
// lie within `near` execution rows of their row.  Each workgroup writes its
// counts (near, all) to part[2 b], part[2 b + 1].
constexpr int kNearLanes = 8;

__global__ void __launch_bounds__(kBT) k_near_count(int32_t n_inst, int32_t nearw, const int64_t* __restrict__ off,
                                                    const int32_t* __restrict__ len,
                                                    const int32_t* __restrict__ col, const int32_t* __restrict__ iperm,
                                                    int64_t* __restrict__ part) {
    __shared__ int64_t red[kBT / kWave];
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t v = (t / kNearLanes) * kSample;
    const int ln = threadIdx.x & (kNearLanes - 1);
    int64_t near = 0, all = 0;
    if (v < n_inst) {
        const int rv = iperm[v];
        const int64_t o = off[v];
        const int l = len[v];
        for (int j = ln; j < l; j += kNearLanes) {
            const int c = col[o + j];
            if (c >= n_inst) continue;
            const int d = iperm[c] - rv;
            near += (d <= nearw && d >= -nearw) ? 1 : 0;
            ++all;
        }
    }
    near = block_sum_i64<kBT>(near, red);
    all = block_sum_i64<kBT>(all, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = near;
        part[2 * blockIdx.x + 1] = all;
    }
}

// The verdict from the workgroups' counts: local when at least a quarter of
// the sampled entries are near their row (or nothing was sampled).
__global__ void __launch_bounds__(kBT) k_loc_flag(const int64_t* __restrict__ part, int32_t nparts,
                                                  int32_t* __restrict__ flag) {
    __shared__ int64_t red[kBT / kWave];
    int64_t near = 0, all = 0;
    for (int b = threadIdx.x; b < nparts; b += kBT) {
        near += part[2 * b];
        all += part[2 * b + 1];
    }
    near = block_sum_i64<kBT>(near, red);
    all = block_sum_i64<kBT>(all, red);
    if (threadIdx.x == 0) flag[0] = (all == 0 || 4 * near >= all) ? 1 : 0;
}

}  // namespace

static void exec_net_copy(Graph& g, int32_t N, hipStream_t s2);

// Two stable LSD passes over np keys (low digit `digit`, then key >> lo_bits
// of that order) into `out`; ties keep node order.
static void sort_keys(Graph& g, DevBuf<int32_t>& key, DevBuf<int32_t>& digit, int32_t np, int lo_bits, int hi_bits,
                      hipStream_t s) {
    DevBuf<int32_t> first, second;
    bucket_sort(g, digit.p, np, 1 << lo_bits, first, g.lay_start, s, false);
    if (lo_bits == kDigitBits)
        hipLaunchKernelGGL(k_high_digit, dim3(grid_for(np, kBT)), dim3(kBT), 0, s, np, key.p, first.p, digit.p);
    else
        hipLaunchKernelGGL(k_hi12, dim3(grid_for(np, kBT)), dim3(kBT), 0, s, np, key.p, first.p, digit.p);
    AHR_LAUNCHED("k_high_digit");
    bucket_sort(g, digit.p, np, 1 << hi_bits, second, g.lay_start, s, false);
    hipLaunchKernelGGL(k_compose, dim3(grid_for(np, kBT)), dim3(kBT), 0, s, np, first.p, second.p, key.p);
    AHR_LAUNCHED("k_compose");
    first.release(s);
    second.release(s);
}

// perm from the sorted order in `key` (instance windows by row length,
// macro pins and stars as sorted), then iperm.
static void finish_perm(Graph& g, DevBuf<int32_t>& key, hipStream_t s) {
    const int32_t n = g.n_inst, N = g.n_tot, np = g.first_mvirt;
    g.perm.ensure(static_cast<size_t>(N) + 1, s);
    hipLaunchKernelGGL(k_window_sort, dim3(grid_for(n, kLenWindow)), dim3(kLenWindow), 0, s, n, key.p, g.net_len.p,
                       g.perm.p);
    AHR_LAUNCHED("k_window_sort");
    if (np > n)
        AHR_HIP(hipMemcpyAsync(g.perm.p + n, key.p + n, static_cast<size_t>(np - n) * sizeof(int32_t),
                               hipMemcpyDeviceToDevice, s));
    g.iperm.ensure(static_cast<size_t>(N) + 1, s);
    hipLaunchKernelGGL(k_iperm, dim3(grid_for(N, kBT)), dim3(kBT), 0, s, g.perm.p, np, N, g.iperm.p);
    AHR_LAUNCHED("k_iperm");
}

// The Hilbert order of the placement's positions.
static void position_order(Graph& g, const float* pos, int32_t ncols, hipStream_t s) {
    const int32_t n = g.n_inst, np = g.first_mvirt;
    DevBuf<int32_t> key, digit;
    key.ensure(static_cast<size_t>(np) + 1, s);
    digit.ensure(static_cast<size_t>(np) + 1, s);
    const float side = static_cast<float>(1 << kGridBits);
    KeyArgs ka;
    ka.pos = pos;
    ka.ncols = ncols;
    ka.n_inst = n;
    ka.first_star = g.first_star;
    ka.first_mvirt = np;
    ka.mpin_pin = g.mpin_pin.p;
    ka.star_net = g.star_net.p;
    ka.net_ptr = g.nl.net_ptr;
    ka.pin_node = g.nl.pin_node;
    ka.pin_node_x = g.pin_node_x.p;
    ka.pin_off = g.nl.pin_off;
    ka.xl = g.nl.die[0];
    ka.yl = g.nl.die[1];
    ka.sx = side / (g.nl.die[2] - g.nl.die[0]);
    ka.sy = side / (g.nl.die[3] - g.nl.die[1]);
    hipLaunchKernelGGL(k_layout_keys, dim3(grid_for(np, kBT)), dim3(kBT), 0, s, ka, key.p, digit.p);
    AHR_LAUNCHED("k_layout_keys");
    // the range bits keep the instances, macro pins and stars in their own id ranges
    sort_keys(g, key, digit, np, kDigitBits, kKeyBits - kDigitBits, s);
    finish_perm(g, key, s);
    key.release(s);
    digit.release(s);
}

// The locality test of the current layout, left on the device (g.loc_flag):
// of a sample of instance rows, the share of instance-to-instance entries
// within n/64 rows (at least 256) of their row.  g.hop_local is read later.
static void locality_begin(Graph& g, hipStream_t s) {
    const int32_t n = g.n_inst;
    const int64_t nt = (static_cast<int64_t>(n) + kSample - 1) / kSample;
    const unsigned blocks = grid_for(nt * kNearLanes, kBT);
    g.loc_part.ensure(2 * static_cast<size_t>(blocks), s);
    g.loc_flag.ensure(1, s);
    const int32_t nearw = n / 64 > 256 ? n / 64 : 256;
    hipLaunchKernelGGL(k_near_count, dim3(blocks), dim3(kBT), 0, s, n, nearw, g.net_off.p, g.net_len.p,
                       g.net_col.p, g.iperm.p, g.loc_part.p);
    AHR_LAUNCHED("k_near_count");
    hipLaunchKernelGGL(k_loc_flag, dim3(1), dim3(kBT), 0, s, g.loc_part.p, static_cast<int32_t>(blocks),
                       g.loc_flag.p);
    AHR_LAUNCHED("k_loc_flag");
    g.hop_local = -1;
}

// Whether the current layout's instance rows sit near their instance
// neighbours (the locality test, read now).
static bool layout_is_local(Graph& g, hipStream_t s) {
    locality_begin(g, s);
    int32_t f = 1;
    read_scalars({g.loc_flag.p}, &f, s);
    g.hop_local = f ? 1 : 0;
    return f != 0;
}

// Cuthill-McKee ranks of the instances (see the file's comment), then the
// netlist order of all instance, macro pin and star rows.
constexpr int kCmMaxLevels = 256;     // beyond that, the rest is appended in id order
constexpr int kCmCheck = 8;           // levels between reads of the level range

static void netlist_order(Graph& g, hipStream_t s) {
    const int32_t n = g.n_inst, np = g.first_mvirt;
    DevBuf<unsigned long long> lk;
    DevBuf<int32_t> rank, order, cnt, scn, bnd;
    const size_t n1 = static_cast<size_t>(n) + 1;
    lk.ensure(n1, s);
    rank.ensure(n1, s);
    order.ensure(n1, s);
    cnt.ensure(n1, s);
    scn.ensure(n1, s);
    bnd.ensure(4, s);
    g.scan_tmp.ensure(scan_tmp_elems(n), s);
    CmArgs a{n, g.net_off.p, g.net_len.p, g.net_col.p, lk.p, rank.p, order.p, cnt.p, scn.p, bnd.p};
    hipLaunchKernelGGL(k_cm_init, dim3(grid_for(n, kBT)), dim3(kBT), 0, s, a);
    AHR_LAUNCHED("k_cm_init");
    hipLaunchKernelGGL(k_cm_start, dim3(grid_for(n, kBT)), dim3(kBT), 0, s, a);
    AHR_LAUNCHED("k_cm_start");
    hipLaunchKernelGGL(k_cm_seed, dim3(1), dim3(1), 0, s, a);
    AHR_LAUNCHED("k_cm_seed");
    for (int k = 0; k < kCmMaxLevels; ++k) {
        hipLaunchKernelGGL(k_cm_expand, dim3(kCmGrid), dim3(256), 0, s, a, k);
        AHR_LAUNCHED("k_cm_expand");
        hipLaunchKernelGGL(k_cm_count, dim3(kCmGrid), dim3(256), 0, s, a, k);
        AHR_LAUNCHED("k_cm_count");
        scan_i32_to_i32(cnt.p, scn.p, n, g.scan_tmp.p, s);
        hipLaunchKernelGGL(k_cm_assign, dim3(kCmGrid), dim3(256), 0, s, a, k);
        AHR_LAUNCHED("k_cm_assign");
        hipLaunchKernelGGL(k_cm_next, dim3(1), dim3(1), 0, s, a);
        AHR_LAUNCHED("k_cm_next");
        if ((k + 1) % kCmCheck == 0) {
            int32_t lh[2];
            read_scalars({bnd.p, bnd.p + 1}, lh, s);
            if (lh[0] == lh[1]) break;
        }
    }
    // the unreached instances after the reached ones
    hipLaunchKernelGGL(k_cm_unplaced, dim3(grid_for(n, kBT)), dim3(kBT), 0, s, n, rank.p, cnt.p);
    AHR_LAUNCHED("k_cm_unplaced");
    scan_i32_to_i32(cnt.p, scn.p, n, g.scan_tmp.p, s);
    hipLaunchKernelGGL(k_cm_append, dim3(grid_for(n, kBT)), dim3(kBT), 0, s, n, cnt.p, scn.p, bnd.p, rank.p);
    AHR_LAUNCHED("k_cm_append");
    lk.release(s);
    order.release(s);
    cnt.release(s);
    scn.release(s);
    bnd.release(s);
    // sort keys: range, then rank (24 bits, two 12-bit passes)
    DevBuf<int32_t> skey, digit;
    skey.ensure(static_cast<size_t>(np) + 1, s);
    digit.ensure(static_cast<size_t>(np) + 1, s);
    hipLaunchKernelGGL(k_cm_keys, dim3(grid_for(n, kBT)), dim3(kBT), 0, s, n, rank.p, skey.p, digit.p);
    AHR_LAUNCHED("k_cm_keys");
    if (np > n) {
        hipLaunchKernelGGL(k_cm_keys_aux, dim3(grid_for(static_cast<int64_t>(np - n) * kWave, kBT)), dim3(kBT), 0,
                           s, n, np, g.first_star, g.net_off.p, g.net_len.p, g.net_col.p, rank.p, skey.p, digit.p);
        AHR_LAUNCHED("k_cm_keys_aux");
    }
    rank.release(s);
    sort_keys(g, skey, digit, np, 12, 12, s);
    finish_perm(g, skey, s);
    skey.release(s);
    digit.release(s);
}

void set_layout(Graph& g, const float* pos, int32_t ncols, hipStream_t s) {
    const int32_t n = g.n_inst, N = g.n_tot, np = g.first_mvirt;
    const uint32_t fl = g.hp.flags;
    const bool cm_ok = n < (1 << 22);           // ranks fit the netlist order's 22-bit keys
    bool netlist = cm_ok && (fl & AHR_LAYOUT_NETLIST);
    bool tested = false;      // the locality test already covers the order taken
    if (!netlist) {
        position_order(g, pos, ncols, s);
        if (cm_ok && (fl & AHR_LAYOUT_AUTO)) {
            tested = layout_is_local(g, s);
            netlist = !tested;
        }
    }
    if (netlist) netlist_order(g, s);
    g.layout_netlist = netlist ? 1 : 0;
    // the hop's launch shape follows the order's locality (AHR_HOP_AUTO); the
    // verdict is read with the first row classes
    if (!tested) locality_begin(g, s);

    DevBuf<int32_t> len;
    len.ensure(static_cast<size_t>(N) + 1, s);
    g.xqdeg.ensure(static_cast<size_t>(N) + 1, s);
    g.xmpin.ensure(static_cast<size_t>(g.first_star - n) + 1, s);
    g.xstar_net.ensure(static_cast<size_t>(np - g.first_star) + 1, s);
    ExecRowArgs ea{N, n, g.first_star, np, g.perm.p, g.net_len.p, g.qdeg.p, g.mpin_pin.p, g.nl.pin_node,
                   g.nl.pin_off, g.star_net.p, len.p, g.xqdeg.p, g.xmpin.p, g.xstar_net.p};
    hipLaunchKernelGGL(k_exec_rows, dim3(grid_for(N, kBT)), dim3(kBT), 0, s, ea);
    AHR_LAUNCHED("k_exec_rows");
    g.xnet_rp.ensure(static_cast<size_t>(N) + 1, s);
    g.scan_tmp.ensure(scan_tmp_elems(N), s);
    scan_i32_to_i32(len.p, g.xnet_rp.p, N, g.scan_tmp.p, s);
    len.release(s);
    g.xnet_ent.ensure(static_cast<size_t>(g.nnz_cap) + 1, s);      // the netlist arrays' bound
    if (g.nnz_cap) {
        // Nothing reads the execution-order entries before the first hop, so
        // their copy runs on the device's side stream, beside the hint build
        // and the degree kernels that follow on s.  Readers take the entries
        // through net_entries(), which orders their stream after the copy.
        if (!g.xnet_fork) AHR_HIP(hipEventCreateWithFlags(&g.xnet_fork, hipEventDisableTiming));
        if (!g.xnet_ready) AHR_HIP(hipEventCreateWithFlags(&g.xnet_ready, hipEventDisableTiming));
        const hipStream_t s2 = side_stream();
        AHR_HIP(hipEventRecord(g.xnet_fork, s));
        AHR_HIP(hipStreamWaitEvent(s2, g.xnet_fork, 0));
        try {
            exec_net_copy(g, N, s2);
        } catch (...) {
            // readers and the destructor still order themselves after what
            // did reach the side stream
            (void)hipEventRecord(g.xnet_ready, s2);
            throw;
        }
        AHR_HIP(hipEventRecord(g.xnet_ready, s2));
        g.xnet_waited = 0;
    }
    g.has_layout = 1;
}

// The execution-order netlist entries: short rows by k_exec_net, long rows
// by k_exec_net_long from a device-built list, all on stream s2.
static void exec_net_copy(Graph& g, int32_t N, hipStream_t s2) {
    hipLaunchKernelGGL(k_exec_net, dim3(grid_for(static_cast<int64_t>(N) * 8, kBT)), dim3(kBT), 0, s2, N,
                       g.perm.p, g.iperm.p, g.net_off.p, g.net_col.p, g.net_q.p, g.xnet_rp.p, g.xnet_ent.p);
    AHR_LAUNCHED("k_exec_net");
    DevBuf<int32_t> flag, rank, rows;
    DevBuf<int64_t> tmp;     // not g.scan_tmp: s uses that meanwhile
    flag.ensure(static_cast<size_t>(N) + 1, s2);
    rank.ensure(static_cast<size_t>(N) + 1, s2);
    tmp.ensure(scan_tmp_elems(N), s2);
    hipLaunchKernelGGL(k_long_flags, dim3(grid_for(N, kBT)), dim3(kBT), 0, s2, N, g.xnet_rp.p, flag.p);
    AHR_LAUNCHED("k_long_flags");
    scan_i32_to_i32(flag.p, rank.p, N, tmp.p, s2);
    rows.ensure(static_cast<size_t>(N) + 1, s2);
    list_rows(flag.p, rank.p, N, rows.p, s2);
    hipLaunchKernelGGL(k_exec_net_long, dim3(kLongRowGrid), dim3(kBT), 0, s2, rows.p, rank.p + N, g.perm.p,
                       g.iperm.p, g.net_off.p, g.net_col.p, g.net_q.p, g.xnet_rp.p, g.xnet_ent.p);
    AHR_LAUNCHED("k_exec_net_long");
    flag.release(s2);
    rank.release(s2);
    rows.release(s2);
    tmp.release(s2);
}

const int2* net_entries(const Graph& g, hipStream_t s) {
    if (g.xnet_ready && !(g.xnet_waited && g.xnet_wait_stream == s)) {
        AHR_HIP(hipStreamWaitEvent(s, g.xnet_ready, 0));
        g.xnet_waited = 1;
        g.xnet_wait_stream = s;
    }
    return g.xnet_ent.p;
}

}  // namespace ahr
