// Area hints of one placement (Section V): bin densities D_b and
// phi_b = 2 sigmoid(mu (D_b - C)) - 1, bin-window edges
// w = -exp(-maxRatio_{i,b}) phi_b baseWeight_i, macro-footprint edges
// w = -exp(-maxRatio_{i,m}) baseWeight_i.  Which entries exist is decided in
// float32 (cell bin, footprint test) and laid out with integer counts and
// scans only, so the structure is exact and run-to-run identical; weights
// are evaluated in float64 and stored as float32, by one function per edge
// kind, so A_ij and A_ji are bit-identical.
#include <algorithm>

#include "ahr_internal.hpp"
#include "device_util.hpp"

namespace ahr {

namespace {

constexpr int kBT = 256;
constexpr int kMaxBins = 16384;
constexpr int kTileIters = 32;                 // bucket sort: 64-lane tiles of 32 x 64 cells
constexpr int kTileCells = kTileIters * kWave;
constexpr double kAreaQ = 268435456.0;         // bin areas in units of 2^-28 (exact integer sums)

struct Grid {
    int nbx, nby;
    float xl32, yl32, bw32, bh32;
    double xl, yl, bw, bh;
    int hx, hy;                                 // window half widths
};

__device__ __forceinline__ int bin_coord(float v, float lo, float w, int nb) {
    float f = floorf((v - lo) / w);
    if (!(f > 0.f)) return 0;                   // also maps NaN to 0
    if (f >= static_cast<float>(nb - 1)) return nb - 1;
    return static_cast<int>(f);
}

__device__ __forceinline__ bool is_std_movable(uint8_t f) { return (f & (AHR_NODE_FIXED | AHR_NODE_MACRO)) == 0; }

// The bin-hint weight of a cell at (x, y) towards bin (bx, by) is
// -exp(-max(rx, ry)) phi_b baseWeight_i, with rx and ry its distances from
// the bin centre in half bin widths.  exp(-max(rx, ry)) is exp(-rx) or
// exp(-ry), whichever argument is the maximum, so a cell's window needs one
// exponential per window column and one per window row.
__device__ __forceinline__ double bin_rx(const Grid& gr, float x, int bx) {
    const double xb = gr.xl + (static_cast<double>(bx) + 0.5) * gr.bw;
    return fabs(static_cast<double>(x) - xb) / (gr.bw / 2);
}

__device__ __forceinline__ double bin_ry(const Grid& gr, float y, int by) {
    const double yb = gr.yl + (static_cast<double>(by) + 0.5) * gr.bh;
    return fabs(static_cast<double>(y) - yb) / (gr.bh / 2);
}

__device__ __forceinline__ float w_bin_of(double rx, double ex, double ry, double ey, double phi_b, double bw_i) {
    const double e = rx > ry ? ex : ey;     // exp(-max(rx, ry))
    return static_cast<float>(-e * phi_b * bw_i);
}

__device__ __forceinline__ bool inside(float x, float y, float4 m) {
    return fabsf(x - m.x) <= m.z && fabsf(y - m.y) <= m.w;
}

__device__ __forceinline__ float w_macro(float x, float y, float4 m, double bw_i) {
    // m.z, m.w are w/2, h/2 (exact halving), so this is |dx| / (w_m / 2)
    double rx = fabs(static_cast<double>(x) - static_cast<double>(m.x)) / static_cast<double>(m.z);
    double ry = fabs(static_cast<double>(y) - static_cast<double>(m.y)) / static_cast<double>(m.w);
    double r = rx > ry ? rx : ry;
    return static_cast<float>(-exp(-r) * bw_i);
}

// Per execution row, once per graph: the cell's fixed-point area times 4
// plus its class (0: not a movable standard cell, 1: movable standard cell
// without nets, 2: movable standard cell with nets, a hint cell), and its
// baseWeight; the per-round kernels then read them in row order.
constexpr int64_t kCellOther = 0, kCellStd = 1, kCellHint = 2;

// One thread per instance, in instance order (coalesced reads), storing to
// its execution row (two scattered stores instead of four scattered loads).
__global__ void k_exec_cells(int32_t n_inst, const int32_t* __restrict__ iperm, const uint8_t* __restrict__ flags,
                             const float* __restrict__ size, const int64_t* __restrict__ qdeg,
                             const double* __restrict__ base_w, int64_t* __restrict__ xcell,
                             double* __restrict__ xbase_w) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_inst) return;
    const int r = iperm[i];
    int64_t c = kCellOther;
    if (is_std_movable(flags[i])) {
        double a = static_cast<double>(size[2 * i]) * static_cast<double>(size[2 * i + 1]);
        int64_t q = static_cast<int64_t>(__builtin_rint(a * kAreaQ));
        c = q * 4 + (qdeg[i] > 0 ? kCellHint : kCellStd);
    }
    xcell[r] = c;
    xbase_w[r] = base_w[i];
}

// Bin of every hint cell (-1 otherwise), indexed by execution row, the
// fixed-point cell area per bin, and the placement in row order (xpos).
// Rows are in spatial order, so a workgroup's cells fall in few bins: areas
// are summed in LDS first (dynamic, nbins counters when nbins <= kLdsBins;
// integer areas, so the sums do not depend on the order).
constexpr int kCellBinRows = 4;      // rows per thread
constexpr int kLdsBins = 4096;

__global__ void __launch_bounds__(kBT) k_cell_bins(Grid gr, const float* __restrict__ pos, int ncols, int32_t n_inst,
                                                   const int32_t* __restrict__ perm,
                                                   const int64_t* __restrict__ xcell, int with_density,
                                                   int32_t* __restrict__ cell_bin, float2* __restrict__ xpos,
                                                   unsigned long long* __restrict__ area_q) {
    extern __shared__ unsigned long long area_lds[];
    if (n_inst <= 0) return;     // (the launch has one workgroup even then; nothing to read)
    const int nbins = gr.nbx * gr.nby;
    const bool lds = nbins <= kLdsBins;
    if (lds && with_density)
        for (int b = threadIdx.x; b < nbins; b += kBT) area_lds[b] = 0ull;
    __syncthreads();
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kBT * kCellBinRows;
    // every row's loads first (the instance, then its position and class),
    // so the thread's kCellBinRows dependent pairs are in flight together;
    // rows past the end read row 0 and are dropped below
    int inst[kCellBinRows];
#pragma unroll
    for (int t = 0; t < kCellBinRows; ++t) {
        const int64_t r = base + static_cast<int64_t>(t) * kBT + threadIdx.x;
        inst[t] = perm[r < n_inst ? r : 0];
    }
    float px[kCellBinRows], py[kCellBinRows];
    int64_t cls[kCellBinRows];
#pragma unroll
    for (int t = 0; t < kCellBinRows; ++t) {
        const int64_t r = base + static_cast<int64_t>(t) * kBT + threadIdx.x;
        px[t] = pos[static_cast<int64_t>(inst[t]) * ncols];
        py[t] = pos[static_cast<int64_t>(inst[t]) * ncols + 1];
        cls[t] = xcell[r < n_inst ? r : 0];
    }
#pragma unroll
    for (int t = 0; t < kCellBinRows; ++t) {
        const int64_t r = base + static_cast<int64_t>(t) * kBT + threadIdx.x;
        if (r >= n_inst) break;
        const float x = px[t], y = py[t];
        xpos[r] = make_float2(x, y);
        const int64_t c = cls[t];
        int b = -1;
        if ((c & 3) != kCellOther) {
            int bx = bin_coord(x, gr.xl32, gr.bw32, gr.nbx);
            int by = bin_coord(y, gr.yl32, gr.bh32, gr.nby);
            int bb = by * gr.nbx + bx;
            if (with_density) {
                unsigned long long q = static_cast<unsigned long long>(c >> 2);
                if (lds) atomicAdd(&area_lds[bb], q);
                else atomicAdd(&area_q[bb], q);
            }
            if ((c & 3) == kCellHint) b = bb;
        }
        cell_bin[r] = b;
    }
    if (lds && with_density) {
        __syncthreads();
        for (int b = threadIdx.x; b < nbins; b += kBT)
            if (area_lds[b]) atomicAdd(&area_q[b], area_lds[b]);
    }
}

// Stable bucket sort, pass 1: hint cells per (bin, tile), bin-major.
__global__ void __launch_bounds__(kWave) k_bucket_count(const int32_t* __restrict__ cell_bin, int32_t n, int nbins,
                                                        int32_t ntiles, int32_t* __restrict__ hist) {
    extern __shared__ int32_t h[];     // nbins counters (dynamic: occupancy follows the key count)
    for (int b = threadIdx.x; b < nbins; b += kWave) h[b] = 0;
    __syncthreads();
    int64_t base = static_cast<int64_t>(blockIdx.x) * kTileCells;
    int key[kTileIters];       // the tile's keys, all loads in flight together
#pragma unroll
    for (int t = 0; t < kTileIters; ++t) {
        int64_t i = base + t * kWave + threadIdx.x;
        key[t] = i < n ? cell_bin[i] : -1;
    }
#pragma unroll
    for (int t = 0; t < kTileIters; ++t)
        if (key[t] >= 0) atomicAdd(&h[key[t]], 1);
    __syncthreads();
    // tile-major: this tile's counters are one contiguous row
    for (int b = threadIdx.x; b < nbins; b += kWave) hist[static_cast<int64_t>(blockIdx.x) * nbins + b] = h[b];
}

// out[c][r] = in[r][c] for an rows x cols int32 matrix, through 32 x 32 LDS tiles.
constexpr int kTr = 32;
__global__ void __launch_bounds__(kTr * 8) k_transpose_i32(const int32_t* __restrict__ in, int64_t rows,
                                                            int64_t cols, int32_t* __restrict__ out) {
    __shared__ int32_t t[kTr][kTr + 1];
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * kTr, r0 = static_cast<int64_t>(blockIdx.y) * kTr;
    const int tx = threadIdx.x % kTr, ty = threadIdx.x / kTr;
    for (int k = ty; k < kTr; k += 8) {
        const int64_t r = r0 + k, c = c0 + tx;
        if (r < rows && c < cols) t[k][tx] = in[r * cols + c];
    }
    __syncthreads();
    for (int k = ty; k < kTr; k += 8) {
        const int64_t c = c0 + k, r = r0 + tx;
        if (r < rows && c < cols) out[c * rows + r] = t[tx][k];
    }
}

// Pass 2: place every hint cell at offset(bin, tile) + rank among the
// tile's earlier cells of the same bin (lanes in id order, tiles in order);
// off is tile-major, like the counts.
__global__ void __launch_bounds__(kWave) k_bucket_scatter(const int32_t* __restrict__ cell_bin, int32_t n, int nbins,
                                                          int bits, int32_t ntiles, const int32_t* __restrict__ off,
                                                          int32_t* __restrict__ out) {
    extern __shared__ int32_t run[];   // nbins cursors (dynamic)
    for (int b = threadIdx.x; b < nbins; b += kWave) run[b] = off[static_cast<int64_t>(blockIdx.x) * nbins + b];
    __syncthreads();
    int l = threadIdx.x;
    uint64_t lt = l ? (~0ull >> (kWave - l)) : 0ull;
    uint64_t gt = (l == kWave - 1) ? 0ull : (~0ull << (l + 1));
    int64_t base = static_cast<int64_t>(blockIdx.x) * kTileCells;
    int key[kTileIters];       // the tile's keys, all loads in flight together
#pragma unroll
    for (int t = 0; t < kTileIters; ++t) {
        int64_t i = base + t * kWave + l;
        key[t] = i < n ? cell_bin[i] : -1;
    }
#pragma unroll
    for (int t = 0; t < kTileIters; ++t) {
        int64_t i = base + t * kWave + l;
        int b = key[t];
        bool valid = b >= 0;
        uint64_t peer = __ballot(valid);
        for (int k = 0; k < bits; ++k) {
            bool bit = valid && ((b >> k) & 1);
            uint64_t m = __ballot(bit);
            peer &= bit ? m : ~m;
        }
        if (valid) {
            int rank = __popcll(peer & lt);
            out[run[b] + rank] = static_cast<int32_t>(i);
        }
        __syncthreads();
        if (valid && (peer & gt) == 0) run[b] += __popcll(peer);
        __syncthreads();
    }
}

__global__ void k_bin_start(const int32_t* __restrict__ off, int nbins, int32_t ntiles,
                            const int32_t* __restrict__ total, int32_t* __restrict__ bin_start) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nbins) bin_start[b] = off[static_cast<int64_t>(b) * ntiles];
    if (b == nbins) bin_start[b] = *total;
}

__device__ __forceinline__ float outward(float c, float h) {
    double v = static_cast<double>(c) + static_cast<double>(h) * (1.0 + 0x1p-20);
    float f = static_cast<float>(v);
    if (h < 0 && static_cast<double>(f) > v) f = nextafterf(f, -INFINITY);
    if (h >= 0 && static_cast<double>(f) < v) f = nextafterf(f, INFINITY);
    return f;
}

// Macro footprint (float32), the bin span of the cells it can hold, and its
// exact area per bin.
__global__ void k_macros(Grid gr, const float* __restrict__ pos, int ncols, const int32_t* __restrict__ macro_ids,
                         int32_t n_macro, const float* __restrict__ size, int with_density, float4* __restrict__ rect,
                         int4* __restrict__ span, unsigned long long* __restrict__ area_q) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_macro) return;
    int m = macro_ids[k];
    float cx = pos[static_cast<int64_t>(m) * ncols], cy = pos[static_cast<int64_t>(m) * ncols + 1];
    float w = size[2 * m], h = size[2 * m + 1];
    float4 r = make_float4(cx, cy, w * 0.5f, h * 0.5f);
    rect[k] = r;
    // Any x with fl(|x - cx|) <= w/2 has |x - cx| < (w/2)(1 + 2^-23), so the
    // span of [cx - (w/2)(1 + 2^-20), cx + (w/2)(1 + 2^-20)], rounded outward
    // to float32, holds the bin of every cell the footprint test accepts
    // (bin_coord is monotone).
    span[k] = make_int4(bin_coord(outward(cx, -r.z), gr.xl32, gr.bw32, gr.nbx),
                        bin_coord(outward(cy, -r.w), gr.yl32, gr.bh32, gr.nby),
                        bin_coord(outward(cx, r.z), gr.xl32, gr.bw32, gr.nbx),
                        bin_coord(outward(cy, r.w), gr.yl32, gr.bh32, gr.nby));
    if (!with_density) return;
    // exact overlap of the footprint with every bin it touches (float64)
    double dcx = cx, dcy = cy, dw = w, dh = h;
    double x0 = dcx - dw / 2, x1 = dcx + dw / 2, y0 = dcy - dh / 2, y1 = dcy + dh / 2;
    int ix0 = static_cast<int>(floor((x0 - gr.xl) / gr.bw)), ix1 = static_cast<int>(floor((x1 - gr.xl) / gr.bw));
    int iy0 = static_cast<int>(floor((y0 - gr.yl) / gr.bh)), iy1 = static_cast<int>(floor((y1 - gr.yl) / gr.bh));
    ix0 = ix0 < 0 ? 0 : ix0;
    iy0 = iy0 < 0 ? 0 : iy0;
    ix1 = ix1 >= gr.nbx ? gr.nbx - 1 : ix1;
    iy1 = iy1 >= gr.nby ? gr.nby - 1 : iy1;
    for (int by = iy0; by <= iy1; ++by) {
        double bl = gr.yl + by * gr.bh, bh_ = gr.yl + (by + 1) * gr.bh;
        double oy = (y1 < bh_ ? y1 : bh_) - (y0 > bl ? y0 : bl);
        if (!(oy > 0)) continue;
        for (int bx = ix0; bx <= ix1; ++bx) {
            double xl_ = gr.xl + bx * gr.bw, xh_ = gr.xl + (bx + 1) * gr.bw;
            double ox = (x1 < xh_ ? x1 : xh_) - (x0 > xl_ ? x0 : xl_);
            if (!(ox > 0)) continue;
            atomicAdd(&area_q[by * gr.nbx + bx],
                      static_cast<unsigned long long>(static_cast<int64_t>(__builtin_rint(oy * ox * kAreaQ))));
        }
    }
}

__global__ void k_phi(int nbins, double bin_area, double cap, double mu, const unsigned long long* __restrict__ area_q,
                      double* __restrict__ phi) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbins) return;
    double D = (static_cast<double>(static_cast<int64_t>(area_q[b])) / kAreaQ) / bin_area;
    phi[b] = 2.0 / (1.0 + exp(-mu * (D - cap))) - 1.0;
}

// Macros whose widened span covers bin b, ascending; pass 1 counts, pass 2 writes.
__global__ void __launch_bounds__(kBT) k_bin_macros(int nbx, const int4* __restrict__ span, int32_t n_macro,
                                                    const int32_t* __restrict__ start, int32_t* __restrict__ cnt,
                                                    int32_t* __restrict__ list) {
    __shared__ int red[kBT / kWave];
    int b = blockIdx.x;
    int bx = b % nbx, by = b / nbx;
    int carry = 0;
    for (int k0 = 0; k0 < n_macro; k0 += kBT) {
        int k = k0 + threadIdx.x;
        bool f = false;
        if (k < n_macro) {
            int4 sp = span[k];
            f = bx >= sp.x && bx <= sp.z && by >= sp.y && by <= sp.w;
        }
        int tot;
        int idx = block_rank<kBT>(f, red, &tot);
        if (list && f) list[start[b] + carry + idx] = k;
        carry += tot;
    }
    if (cnt && threadIdx.x == 0) cnt[b] = carry;
}

struct HintArgs {
    Grid gr;
    const float* pos;
    int ncols;
    int32_t n_inst, n_macro, nbins;
    int32_t first_mvirt, first_bvirt;
    int macro_hints, bin_hints;
    const int32_t* perm;          // execution row -> instance
    const int32_t* cell_bin;      // by execution row
    const int32_t* bin_start;
    const int32_t* bin_cells;     // execution rows by bin
    const int32_t* bm_start;
    const int32_t* bm_list;
    const float4* rect;
    const int4* span;
    const double* phi;
    const double* base_w;         // by instance
    const float2* xpos;           // by execution row
    const double* xbase_w;        // by execution row
    double* habs;                 // by execution row: sum of |weight| of the cell's hint entries
    float* hsg;                   // by execution row: their signed sum
    double prune_tau;             // bin edges of salience exp(-maxRatio) |phi_b| below it are dropped (0: none)
    // Pruning decided in the count pass (windows of at most 64 slots): the
    // kept window slots of each cell (bit j: slot j of the cell's own window,
    // row-major), the kept cells per (bin, slot), and the cells' macro counts.
    unsigned long long* keep_mask;
    const int32_t* kept;
    const int32_t* nmac;
};

// A cell's window slot j (row-major over its own window) holds bin
// (bx + j % ww - hx, by + j / ww - hy); seen from that bin, the cell's bin is
// slot wslots - 1 - j of the bin's window.
__device__ __forceinline__ bool keep_bin_edge(double rx, double ex, double ry, double ey, double phi_b, double tau) {
    return (rx > ry ? ex : ey) * fabs(phi_b) >= tau;
}

__device__ __forceinline__ void window(const Grid& gr, int b, int& x0, int& x1, int& y0, int& y1) {
    int bx = b % gr.nbx, by = b / gr.nbx;
    x0 = bx - gr.hx < 0 ? 0 : bx - gr.hx;
    x1 = bx + gr.hx >= gr.nbx ? gr.nbx - 1 : bx + gr.hx;
    y0 = by - gr.hy < 0 ? 0 : by - gr.hy;
    y1 = by + gr.hy >= gr.nby ? gr.nby - 1 : by + gr.hy;
}

// Per hint cell (execution row): the macros whose footprint holds it and the
// size of its bin window.  With `pairs`, also lists its (row, macro) pairs
// at pair_off[r] in ascending macro order.
__global__ void __launch_bounds__(kBT) k_cell_count(HintArgs a, int32_t* __restrict__ nmac,
                                                    int32_t* __restrict__ nwin, const int32_t* __restrict__ pair_off,
                                                    int32_t* __restrict__ pair_row, int32_t* __restrict__ pair_mac) {
    int64_t r = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x;
    if (r >= a.n_inst) return;
    int b = a.cell_bin[r];
    if (b < 0) {
        if (nmac) nmac[r] = 0, nwin[r] = 0;
        return;
    }
    int n = 0;
    if (a.macro_hints) {
        const float2 xy = a.xpos[r];
        const float x = xy.x, y = xy.y;
        int o = pair_row ? pair_off[r] : 0;
        for (int t = a.bm_start[b]; t < a.bm_start[b + 1]; ++t) {
            int k = a.bm_list[t];
            if (inside(x, y, a.rect[k])) {
                if (pair_row) {
                    pair_row[o + n] = static_cast<int32_t>(r);
                    pair_mac[o + n] = k;
                }
                ++n;
            }
        }
    }
    if (nmac) {
        nmac[r] = n;
        int x0, x1, y0, y1;
        window(a.gr, b, x0, x1, y0, y1);
        if (a.keep_mask) {
            // the salience test of every window bin, as the fill takes it
            const float2 xy = a.xpos[r];
            const int ww = 2 * a.gr.hx + 1, bx = b % a.gr.nbx, by = b / a.gr.nbx;
            unsigned long long m = 0ull;
            for (int ty = y0; ty <= y1; ++ty) {
                const double ry = bin_ry(a.gr, xy.y, ty), ey = exp(-ry);
                for (int tx = x0; tx <= x1; ++tx) {
                    const double rx = bin_rx(a.gr, xy.x, tx);
                    if (keep_bin_edge(rx, exp(-rx), ry, ey, a.phi[ty * a.gr.nbx + tx], a.prune_tau))
                        m |= 1ull << ((ty - by + a.gr.hy) * ww + (tx - bx + a.gr.hx));
                }
            }
            a.keep_mask[r] = m;
            nwin[r] = __popcll(m);
        } else {
            nwin[r] = a.bin_hints ? (x1 - x0 + 1) * (y1 - y0 + 1) : 0;
        }
    }
}

// Pruned bin rows are built over tiles: each bin's cells (bin_cells order)
// cut into runs of kBT, tile_start[b] the first tile of bin b.  The tile of
// workgroup `tile`, or false past the last one.
__device__ __forceinline__ bool tile_of(const int32_t* tile_start, int nbins, int tile, int& b, int& k) {
    if (tile >= tile_start[nbins]) return false;
    int lo = 0, hi = nbins - 1;          // the last bin whose first tile is <= tile
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tile_start[mid] <= tile) lo = mid; else hi = mid - 1;
    }
    b = lo;
    k = tile - tile_start[lo];
    return true;
}

__global__ void k_bin_tile_counts(const int32_t* __restrict__ bin_start, int nbins, int32_t* __restrict__ ntiles) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nbins) ntiles[b] = (bin_start[b + 1] - bin_start[b] + kBT - 1) / kBT;
}

// tcnt[tile * wslots + j]: the tile's cells keeping window slot j (wave
// ballots, integer sums).
__global__ void __launch_bounds__(kBT) k_tile_keep_counts(HintArgs a, const int32_t* __restrict__ tile_start,
                                                          int wslots, int32_t* __restrict__ tcnt) {
    __shared__ int wtot[kBT / kWave][64];
    int b, k;
    if (!tile_of(tile_start, a.nbins, blockIdx.x, b, k)) return;
    const int t = a.bin_start[b] + k * kBT + static_cast<int>(threadIdx.x);
    const unsigned long long m = t < a.bin_start[b + 1] ? a.keep_mask[a.bin_cells[t]] : 0ull;
    for (int j = 0; j < wslots; ++j) {
        const unsigned long long bal = __ballot((m >> j) & 1ull);
        if (lane_id() == 0) wtot[wave_id()][j] = __popcll(bal);
    }
    __syncthreads();
    if (threadIdx.x < wslots) {
        int n = 0;
        for (int w = 0; w < kBT / kWave; ++w) n += wtot[w][threadIdx.x];
        tcnt[static_cast<int64_t>(blockIdx.x) * wslots + threadIdx.x] = n;
    }
}

// Per (bin, slot): each tile's carry (kept cells of the bin's earlier tiles)
// in place of its count, and kept[b * wslots + j], the bin's total.
__global__ void k_tile_carry(const int32_t* __restrict__ tile_start, int nbins, int wslots,
                             int32_t* __restrict__ tcnt, int32_t* __restrict__ kept) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= static_cast<int64_t>(nbins) * wslots) return;
    const int b = static_cast<int>(i / wslots), j = static_cast<int>(i % wslots);
    int acc = 0;
    for (int t = tile_start[b]; t < tile_start[b + 1]; ++t) {
        const int64_t q = static_cast<int64_t>(t) * wslots + j;
        const int c = tcnt[q];
        tcnt[q] = acc;
        acc += c;
    }
    kept[i] = acc;
}

// The three row-count passes in one launch (they write disjoint rows of
// cnt): cell rows, then macro rows (when mb > 0 workgroups), then bin rows.
__global__ void k_hint_row_counts(HintArgs a, int32_t n_inst, const int32_t* __restrict__ nmac,
                                  const int32_t* __restrict__ nwin, int32_t n_macro, int32_t first_mvirt,
                                  const int32_t* __restrict__ mstart, int32_t cb, int32_t mb,
                                  int32_t* __restrict__ cnt) {
    const int32_t b = static_cast<int32_t>(blockIdx.x);
    const int64_t t = static_cast<int64_t>(threadIdx.x);
    if (b < cb) {
        const int64_t r = static_cast<int64_t>(b) * kBT + t;
        if (r < n_inst) cnt[r] = nmac[r] + nwin[r];
    } else if (b < cb + mb) {
        const int64_t k = static_cast<int64_t>(b - cb) * kBT + t;
        if (k < n_macro) cnt[first_mvirt + k] = mstart[k + 1] - mstart[k];
    } else {
        const int64_t bin = static_cast<int64_t>(b - cb - mb) * kBT + t;
        if (bin >= a.nbins) return;
        int x0, x1, y0, y1;
        window(a.gr, static_cast<int>(bin), x0, x1, y0, y1);
        int n = 0;
        const int ww = 2 * a.gr.hx + 1, wslots = ww * (2 * a.gr.hy + 1);
        const int tbx = static_cast<int>(bin % a.gr.nbx), tby = static_cast<int>(bin / a.gr.nbx);
        for (int by = y0; by <= y1; ++by)
            for (int bx = x0; bx <= x1; ++bx) {
                const int bb = by * a.gr.nbx + bx;
                if (a.kept)     // the cells of bb keeping their edge to this bin
                    n += a.kept[static_cast<int64_t>(bb) * wslots + (tby - by + a.gr.hy) * ww + (tbx - bx + a.gr.hx)];
                else
                    n += a.bin_start[bb + 1] - a.bin_start[bb];
            }
        cnt[a.first_bvirt + bin] = n;
    }
}

// Cell rows: macro entries (ascending macro) then window bins (row-major).
// Each bin entry is also written, with the same float, into the bin's own
// row: bin row b lists the cells of its window bins slot by slot (row-major),
// ascending execution rows within a slot; wpre[b][slot] is the slot's offset
// and rank[r] the cell's position in its bin's list.  One thread per cell:
// the bin-row stores of a wave are then consecutive slots of one bin row.
// The workgroup's cell rows are one contiguous range of entries; they are
// assembled in LDS (up to kFillCap entries; any further ones are stored
// directly) and stored with coalesced writes.  Each cell's sums of |w| and
// of w over its hint entries (its hint degree and the signed hint sum) are
// formed on the way, in float64.
constexpr int kFillCap = 16 * kBT;
constexpr int kWinCols = 5;      // windows up to this wide keep their column terms in registers

__global__ void __launch_bounds__(kBT) k_cell_fill(HintArgs a, const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ pair_off,
                                                   const int32_t* __restrict__ pair_mac,
                                                   const int32_t* __restrict__ rank, const int32_t* __restrict__ wpre,
                                                   int2* __restrict__ ent) {
    __shared__ int2 stage[kFillCap];
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kBT;
    const int64_t r = r0 + threadIdx.x;
    const int64_t rend = r0 + kBT < a.n_inst ? r0 + kBT : a.n_inst;
    const int64_t e0 = rp[r0], e1 = rp[rend];       // the workgroup's cell-row entries
    double ha = 0.0, hs = 0.0;
    if (r < a.n_inst) {
        const int b = a.cell_bin[r];
        if (b >= 0) {
            const float2 xy = a.xpos[r];
            const float x = xy.x, y = xy.y;
            const double bwi = a.xbase_w[r];
            const int64_t o = rp[r] - e0;
            int n = 0;
            auto put = [&](int2 v) {
                const int64_t k = o + n++;
                if (k < kFillCap)
                    stage[k] = v;
                else
                    ent[e0 + k] = v;
            };
            for (int p = pair_off[r]; p < pair_off[r + 1]; ++p) {
                int k = pair_mac[p];
                const float wm = w_macro(x, y, a.rect[k], bwi);
                ha += fabs(static_cast<double>(wm));
                hs += static_cast<double>(wm);
                put(make_int2(a.first_mvirt + k, f_bits(wm)));
            }
            if (a.bin_hints) {
                const int ww = 2 * a.gr.hx + 1, wh = 2 * a.gr.hy + 1;
                const int bx = b % a.gr.nbx, by = b / a.gr.nbx;
                const int my = rank[r] - a.bin_start[b];
                int x0, x1, y0, y1;
                window(a.gr, b, x0, x1, y0, y1);
                const unsigned long long kmask = a.keep_mask ? a.keep_mask[r] : 0ull;
                auto bin_entry = [&](int tx, int ty, double rx, double ex, double ry, double ey) {
                    const int bb = ty * a.gr.nbx + tx;
                    if (a.keep_mask) {
                        // pruning decided by the count pass: kept edges only, and the
                        // bin rows are written by k_bin_side_fill
                        if (!((kmask >> ((ty - by + a.gr.hy) * ww + (tx - bx + a.gr.hx))) & 1ull)) return;
                        const float wb = w_bin_of(rx, ex, ry, ey, a.phi[bb], bwi);
                        ha += fabs(static_cast<double>(wb));
                        hs += static_cast<double>(wb);
                        put(make_int2(a.first_bvirt + bb, f_bits(wb)));
                        return;
                    }
                    const int slot = (by - ty + a.gr.hy) * ww + (bx - tx + a.gr.hx);
                    const int64_t q = rp[a.first_bvirt + bb] + wpre[static_cast<int64_t>(bb) * ww * wh + slot] + my;
                    if (a.prune_tau > 0.0 && !keep_bin_edge(rx, ex, ry, ey, a.phi[bb], a.prune_tau)) {
                        // below the salience threshold: both sides become holes that
                        // the compaction removes
                        put(make_int2(-1, 0));
                        ent[q] = make_int2(-1, 0);
                        return;
                    }
                    const float wb = w_bin_of(rx, ex, ry, ey, a.phi[bb], bwi);
                    ha += fabs(static_cast<double>(wb));
                    hs += static_cast<double>(wb);
                    const int w = f_bits(wb);
                    put(make_int2(a.first_bvirt + bb, w));
                    // (q: the slot of this cell's bin inside the window of bb)
                    ent[q] = make_int2(static_cast<int>(r), w);
                };
                const int nx = x1 - x0 + 1;
                if (nx <= kWinCols) {
                    // the window's column distances and exponentials, once
                    double rxs[kWinCols], exs[kWinCols];
#pragma unroll
                    for (int i = 0; i < kWinCols; ++i) {
                        rxs[i] = bin_rx(a.gr, x, i < nx ? x0 + i : x0);
                        exs[i] = i < nx ? exp(-rxs[i]) : 0.0;
                    }
                    for (int ty = y0; ty <= y1; ++ty) {
                        const double ry = bin_ry(a.gr, y, ty), ey = exp(-ry);
#pragma unroll
                        for (int i = 0; i < kWinCols; ++i)
                            if (i < nx) bin_entry(x0 + i, ty, rxs[i], exs[i], ry, ey);
                    }
                } else {
                    for (int ty = y0; ty <= y1; ++ty) {
                        const double ry = bin_ry(a.gr, y, ty), ey = exp(-ry);
                        for (int tx = x0; tx <= x1; ++tx) {
                            const double rx = bin_rx(a.gr, x, tx);
                            bin_entry(tx, ty, rx, exp(-rx), ry, ey);
                        }
                    }
                }
            }
        }
    }
    if (r < a.n_inst) {
        a.habs[r] = ha;
        a.hsg[r] = static_cast<float>(hs);
    }
    __syncthreads();
    const int64_t nst = e1 - e0 < kFillCap ? e1 - e0 : kFillCap;
    for (int64_t k = threadIdx.x; k < nst; k += kBT) ent[e0 + k] = stage[k];
}

// The bin rows of a pruned graph, one tile of a bin's cells per workgroup:
// a cell's kept window slot j goes to bin row bb (the slot's bin), at that
// row's offset for this bin's slot, after the kept cells of the bin's
// earlier tiles (carry) and of this tile before it (wave ballots, the waves
// in order), i.e. in ascending execution rows.  The weight is the one the
// cell's own row holds for bb.
__global__ void __launch_bounds__(kBT) k_bin_side_fill(HintArgs a, const int32_t* __restrict__ tile_start,
                                                       const int32_t* __restrict__ carry,
                                                       const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ wpre, int2* __restrict__ ent) {
    __shared__ int wtot[kBT / kWave][64];
    int b, kt;
    if (!tile_of(tile_start, a.nbins, blockIdx.x, b, kt)) return;
    const int ww = 2 * a.gr.hx + 1, wslots = ww * (2 * a.gr.hy + 1);
    const int bx = b % a.gr.nbx, by = b / a.gr.nbx;
    const int l = lane_id(), wv = wave_id();
    const unsigned long long lt = l ? (~0ull >> (kWave - l)) : 0ull;
    const int t = a.bin_start[b] + kt * kBT + static_cast<int>(threadIdx.x);
    const int r = t < a.bin_start[b + 1] ? a.bin_cells[t] : -1;
    const unsigned long long m = r >= 0 ? a.keep_mask[r] : 0ull;
    for (int j = 0; j < wslots; ++j) {
        const unsigned long long bal = __ballot((m >> j) & 1ull);
        if (l == 0) wtot[wv][j] = __popcll(bal);
    }
    __syncthreads();
    const int64_t own = r >= 0 ? static_cast<int64_t>(rp[r]) + a.nmac[r] : 0;
    const int32_t* c0 = carry + static_cast<int64_t>(blockIdx.x) * wslots;
    for (int j = 0; j < wslots; ++j) {
        const bool set = (m >> j) & 1ull;
        const unsigned long long bal = __ballot(set);    // (every lane takes part)
        if (set) {
            // the bin's kept cells before this one: earlier tiles, earlier
            // waves of this tile, earlier lanes of this wave
            int rank = c0[j] + __popcll(bal & lt);
            for (int w = 0; w < wv; ++w) rank += wtot[w][j];
            const int tx = bx + j % ww - a.gr.hx, ty = by + j / ww - a.gr.hy;
            const int bb = ty * a.gr.nbx + tx;
            const int k = __popcll(m & ((1ull << j) - 1ull));   // this edge's place among the cell's
            const int64_t q = static_cast<int64_t>(rp[a.first_bvirt + bb]) +
                              wpre[static_cast<int64_t>(bb) * wslots + (wslots - 1 - j)] + rank;
            ent[q] = make_int2(r, ent[own + k].y);
        }
    }
}

__global__ void k_bin_rank(int32_t n, const int32_t* __restrict__ bin_cells, int32_t* __restrict__ rank) {
    int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < n) rank[bin_cells[t]] = static_cast<int32_t>(t);
}

// wpre[b][slot]: entries of bin row b before window slot `slot` (row-major,
// out-of-grid slots empty).
__global__ void k_window_prefix(HintArgs a, int32_t* __restrict__ wpre) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.nbins) return;
    const int ww = 2 * a.gr.hx + 1, wh = 2 * a.gr.hy + 1;
    const int bx = b % a.gr.nbx, by = b / a.gr.nbx;
    int acc = 0;
    for (int w = 0; w < ww * wh; ++w) {
        wpre[static_cast<int64_t>(b) * ww * wh + w] = acc;
        int tx = bx + w % ww - a.gr.hx, ty = by + w / ww - a.gr.hy;
        if (tx < 0 || tx >= a.gr.nbx || ty < 0 || ty >= a.gr.nby) continue;
        int bb = ty * a.gr.nbx + tx;
        acc += a.kept ? a.kept[static_cast<int64_t>(bb) * ww * wh + (ww * wh - 1 - w)]
                      : a.bin_start[bb + 1] - a.bin_start[bb];
    }
}

// Macro virtual rows: the transpose of the cell->macro pairs (pairs grouped
// by macro, ascending row); each weight is the cell-side entry's value.
__global__ void k_macro_fill(int32_t n_pairs, int32_t first_mvirt, const int32_t* __restrict__ mlist,
                             const int32_t* __restrict__ mstart, const int32_t* __restrict__ pair_row,
                             const int32_t* __restrict__ pair_mac, const int32_t* __restrict__ pair_off,
                             const int32_t* __restrict__ rp, int2* __restrict__ ent) {
    int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n_pairs) return;
    int p = mlist[t];
    int row = pair_row[p];
    int k = pair_mac[p];
    int w = ent[rp[row] + (p - pair_off[row])].y;
    ent[rp[first_mvirt + k] + (t - mstart[k])] = make_int2(row, w);
}

__global__ void k_copy_u64(const unsigned long long* __restrict__ src, unsigned long long* __restrict__ dst,
                           int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ void k_add_u64(const unsigned long long* __restrict__ src, unsigned long long* __restrict__ dst,
                          int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) dst[i] += src[i];
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

}  // namespace

int32_t bucket_sort(const int32_t* key, int32_t n, int nkeys, DevBuf<int32_t>& list, DevBuf<int32_t>& start,
                    DevBuf<int32_t>& i32a, DevBuf<int32_t>& i32b, DevBuf<int64_t>& scan_tmp, hipStream_t s,
                    bool read_total) {
    if (nkeys > kMaxBins) throw Error{AHR_EUNSUPPORTED, "too many buckets (at most 16384 bins or macros)"};
    list.ensure(static_cast<size_t>(n) + 1, s);
    start.ensure(static_cast<size_t>(nkeys) + 1, s);
    if (n == 0) {
        fill_i32(start.p, nkeys + 1, 0, s);
        return 0;
    }
    int32_t ntiles = static_cast<int32_t>((static_cast<int64_t>(n) + kTileCells - 1) / kTileCells);
    int64_t hn = static_cast<int64_t>(nkeys) * ntiles;
    i32a.ensure(static_cast<size_t>(hn) + 1, s);
    i32b.ensure(static_cast<size_t>(hn) + 1, s);
    const size_t lds = static_cast<size_t>(nkeys) * sizeof(int32_t);
    // counts tile-major (i32a) -> bucket-major (i32b) -> exclusive scan in
    // bucket-then-tile order (i32a, total at [hn]) -> tile-major offsets (i32b)
    hipLaunchKernelGGL(k_bucket_count, dim3(ntiles), dim3(kWave), lds, s, key, n, nkeys, ntiles, i32a.p);
    AHR_LAUNCHED("k_bucket_count");
    hipLaunchKernelGGL(k_transpose_i32, dim3((nkeys + kTr - 1) / kTr, (ntiles + kTr - 1) / kTr), dim3(kTr * 8), 0, s,
                       i32a.p, static_cast<int64_t>(ntiles), static_cast<int64_t>(nkeys), i32b.p);
    AHR_LAUNCHED("k_transpose_i32");
    scan_tmp.ensure(scan_tmp_elems(hn), s);
    scan_i32_to_i32(i32b.p, i32a.p, hn, scan_tmp.p, s);
    hipLaunchKernelGGL(k_transpose_i32, dim3((ntiles + kTr - 1) / kTr, (nkeys + kTr - 1) / kTr), dim3(kTr * 8), 0, s,
                       i32a.p, static_cast<int64_t>(nkeys), static_cast<int64_t>(ntiles), i32b.p);
    AHR_LAUNCHED("k_transpose_i32");
    int bits = 0;
    while ((1 << bits) < nkeys) ++bits;
    hipLaunchKernelGGL(k_bucket_scatter, dim3(ntiles), dim3(kWave), lds, s, key, n, nkeys, bits, ntiles, i32b.p,
                       list.p);
    AHR_LAUNCHED("k_bucket_scatter");
    hipLaunchKernelGGL(k_bin_start, dim3(grid_for(nkeys + 1, kBT)), dim3(kBT), 0, s, i32a.p, nkeys, ntiles,
                       i32a.p + hn, start.p);
    AHR_LAUNCHED("k_bin_start");
    if (!read_total) return -1;
    return read_i32(start.p + nkeys, s);
}

int32_t bucket_sort(Graph& g, const int32_t* key, int32_t n, int nkeys, DevBuf<int32_t>& list,
                    DevBuf<int32_t>& start, hipStream_t s, bool read_total) {
    return bucket_sort(key, n, nkeys, list, start, g.i32a, g.i32b, g.scan_tmp, s, read_total);
}

namespace {

int window_half(float ratio, int nb) {
    // n = max(1, floor(ratio * numBin)) in float32; the window spans +-floor(n/2)
    float p = ratio * static_cast<float>(nb);
    int n = static_cast<int>(floorf(p));
    if (n < 1) n = 1;
    return n / 2;
}

}  // namespace

// Salience pruning: entries marked with column -1 by the fill are removed,
// every row keeping its order.  keep[e] = 1 for a kept entry below the
// entry count (read on the device), 0 otherwise.
__global__ void k_keep_flags(const int2* __restrict__ ent, const int32_t* __restrict__ nnz, int64_t cap,
                             int32_t* __restrict__ keep) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x;
    if (e < cap) keep[e] = e < *nnz && ent[e].x >= 0 ? 1 : 0;
}

__global__ void k_compact(const int2* __restrict__ ent, const int32_t* __restrict__ nnz,
                          const int32_t* __restrict__ keep, const int32_t* __restrict__ pos,
                          const int32_t* __restrict__ rp, int32_t n_rows, int2* __restrict__ out,
                          int32_t* __restrict__ out_rp, int64_t cap) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x;
    if (e < cap && e < *nnz && keep[e]) out[pos[e]] = ent[e];
    if (e <= n_rows) out_rp[e] = pos[rp[e]];
}

void prune_hints(Graph& g, int64_t cap, hipStream_t s) {
    const int32_t N = g.n_tot;
    const int64_t n = cap > N + 1 ? cap : N + 1;
    DevBuf<int32_t> keep, pos, rp;
    DevBuf<int2> ent;
    keep.ensure(static_cast<size_t>(cap) + 1, s);
    pos.ensure(static_cast<size_t>(cap) + 1, s);
    rp.ensure(static_cast<size_t>(N) + 1, s);
    ent.ensure(static_cast<size_t>(cap) + 1, s);
    hipLaunchKernelGGL(k_keep_flags, dim3(grid_for(cap, kBT)), dim3(kBT), 0, s, g.xhint_ent.p, g.xhint_rp.p + N, cap,
                       keep.p);
    AHR_LAUNCHED("k_keep_flags");
    g.scan_tmp.ensure(scan_tmp_elems(cap), s);
    scan_i32_to_i32(keep.p, pos.p, cap, g.scan_tmp.p, s);
    hipLaunchKernelGGL(k_compact, dim3(grid_for(n, kBT)), dim3(kBT), 0, s, g.xhint_ent.p, g.xhint_rp.p + N, keep.p,
                       pos.p, g.xhint_rp.p, N, ent.p, rp.p, cap);
    AHR_LAUNCHED("k_compact");
    std::swap(g.xhint_ent.p, ent.p);
    std::swap(g.xhint_ent.n, ent.n);
    std::swap(g.xhint_rp.p, rp.p);
    std::swap(g.xhint_rp.n, rp.n);
    keep.release(s);
    pos.release(s);
    rp.release(s);
    ent.release(s);
    g.nnz_hint = -1;
}

void build_hints(Graph& g, const float* pos, int32_t ncols, hipStream_t s, bool macros_unchanged) {
    ProfScope ps(kStageHints, s);
    const ahr_hint_params& hp = g.hp;
    const int macro_hints = (hp.flags & AHR_MACRO_HINTS) ? 1 : 0;
    const int bin_hints = (hp.flags & AHR_BIN_HINTS) ? 1 : 0;
    const int32_t N = g.n_tot, n_inst = g.n_inst;
    if (!g.has_layout) set_layout(g, pos, ncols, s);
    g.hint_cnt.ensure(static_cast<size_t>(N) + 1, s);
    g.xhint_rp.ensure(static_cast<size_t>(N) + 1, s);
    fill_i32(g.hint_cnt.p, N + 1, 0, s);
    g.hint_version++;
    g.has_hints = 1;
    if (!macro_hints && !bin_hints) {
        fill_i32(g.xhint_rp.p, N + 1, 0, s);
        g.nnz_hint = 0;
        g.n_hint_cells = 0;
        g.xhint_ent.ensure(1, s);
        AHR_HIP(hipStreamSynchronize(s));
        return;
    }

    Grid gr;
    gr.nbx = hp.nbx;
    gr.nby = hp.nby;
    gr.xl32 = g.nl.die[0];
    gr.yl32 = g.nl.die[1];
    gr.bw32 = (g.nl.die[2] - g.nl.die[0]) / static_cast<float>(hp.nbx);
    gr.bh32 = (g.nl.die[3] - g.nl.die[1]) / static_cast<float>(hp.nby);
    gr.xl = g.nl.die[0];
    gr.yl = g.nl.die[1];
    gr.bw = (static_cast<double>(g.nl.die[2]) - static_cast<double>(g.nl.die[0])) / hp.nbx;
    gr.bh = (static_cast<double>(g.nl.die[3]) - static_cast<double>(g.nl.die[1])) / hp.nby;
    gr.hx = window_half(hp.detection_ratio, hp.nbx);
    gr.hy = window_half(hp.detection_ratio, hp.nby);
    const int nbins = hp.nbx * hp.nby;

    // 1. cell bins (execution rows), cell areas, positions in row order
    if (!g.has_xcell) {
        g.xcell.ensure(static_cast<size_t>(n_inst) + 1, s);
        g.xbase_w.ensure(static_cast<size_t>(n_inst) + 1, s);
        hipLaunchKernelGGL(k_exec_cells, dim3(grid_for(n_inst, kBT)), dim3(kBT), 0, s, n_inst, g.iperm.p,
                           g.nl.node_flags, g.nl.node_size, g.qdeg.p, g.base_w.p, g.xcell.p, g.xbase_w.p);
        AHR_LAUNCHED("k_exec_cells");
        g.has_xcell = 1;
    }
    g.xpos.ensure(static_cast<size_t>(n_inst) + 1, s);
    g.cell_bin.ensure(static_cast<size_t>(n_inst) + 1, s);
    g.bin_area_q.ensure(static_cast<size_t>(nbins) + 1, s);
    // With every macro fixed and where the last call put them, their
    // footprints, spans, per-bin areas and bin lists are those of that call.
    const bool reuse = macros_unchanged && g.macro_cache && g.n_movable_macro == 0;
    g.macro_cache = 0;
    if (reuse && bin_hints) {     // the density starts from the macros' areas
        hipLaunchKernelGGL(k_copy_u64, dim3(grid_for(nbins, kBT)), dim3(kBT), 0, s,
                           reinterpret_cast<const unsigned long long*>(g.macro_area_q.p),
                           reinterpret_cast<unsigned long long*>(g.bin_area_q.p), static_cast<int64_t>(nbins));
        AHR_LAUNCHED("k_copy_u64");
    } else {
        hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(nbins, kBT)), dim3(kBT), 0, s,
                           reinterpret_cast<unsigned long long*>(g.bin_area_q.p), static_cast<int64_t>(nbins));
        AHR_LAUNCHED("k_fill_u64");
    }
    const size_t bins_lds = nbins <= kLdsBins ? static_cast<size_t>(nbins) * sizeof(unsigned long long) : 0;
    hipLaunchKernelGGL(k_cell_bins, dim3(grid_for(n_inst, kBT * kCellBinRows)), dim3(kBT), bins_lds, s, gr, pos, ncols,
                       n_inst, g.perm.p, g.xcell.p, bin_hints, g.cell_bin.p, g.xpos.p,
                       reinterpret_cast<unsigned long long*>(g.bin_area_q.p));
    AHR_LAUNCHED("k_cell_bins");

    // 2. hint cells grouped by bin, ascending execution rows (stable bucket sort)
    bucket_sort(g, g.cell_bin.p, n_inst, nbins, g.bin_cells, g.bin_start, s, false);

    // 3. macros: footprints, spans, areas; phi
    const int32_t n_macro = g.n_macro;
    g.macro_rect.ensure(static_cast<size_t>(n_macro) + 1, s);
    g.macro_span.ensure(static_cast<size_t>(n_macro) + 1, s);
    if (n_macro && !reuse) {
        // the macros' areas go to macro_area_q (kept), then into the density
        g.macro_area_q.ensure(static_cast<size_t>(nbins) + 1, s);
        hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(nbins, kBT)), dim3(kBT), 0, s,
                           reinterpret_cast<unsigned long long*>(g.macro_area_q.p), static_cast<int64_t>(nbins));
        AHR_LAUNCHED("k_fill_u64");
        hipLaunchKernelGGL(k_macros, dim3(grid_for(n_macro, kBT)), dim3(kBT), 0, s, gr, pos, ncols, g.macro_ids.p,
                           n_macro, g.nl.node_size, bin_hints, g.macro_rect.p, g.macro_span.p,
                           reinterpret_cast<unsigned long long*>(g.macro_area_q.p));
        AHR_LAUNCHED("k_macros");
        if (bin_hints) {
            hipLaunchKernelGGL(k_add_u64, dim3(grid_for(nbins, kBT)), dim3(kBT), 0, s,
                               reinterpret_cast<const unsigned long long*>(g.macro_area_q.p),
                               reinterpret_cast<unsigned long long*>(g.bin_area_q.p), static_cast<int64_t>(nbins));
            AHR_LAUNCHED("k_add_u64");
        }
    }
    g.phi.ensure(static_cast<size_t>(nbins) + 1, s);
    if (bin_hints) {
        hipLaunchKernelGGL(k_phi, dim3(grid_for(nbins, kBT)), dim3(kBT), 0, s, nbins, gr.bw * gr.bh,
                           static_cast<double>(hp.bin_capacity), static_cast<double>(hp.mu),
                           reinterpret_cast<const unsigned long long*>(g.bin_area_q.p), g.phi.p);
        AHR_LAUNCHED("k_phi");
    }

    // 4. macros per bin
    const int use_macros = macro_hints && n_macro > 0;
    g.bm_start.ensure(static_cast<size_t>(nbins) + 1, s);
    if (use_macros && !reuse) {
        DevBuf<int32_t> bmc;
        bmc.ensure(static_cast<size_t>(nbins) + 1, s);
        hipLaunchKernelGGL(k_bin_macros, dim3(nbins), dim3(kBT), 0, s, hp.nbx, g.macro_span.p, n_macro,
                           static_cast<const int32_t*>(nullptr), bmc.p, static_cast<int32_t*>(nullptr));
        AHR_LAUNCHED("k_bin_macros count");
        g.scan_tmp.ensure(scan_tmp_elems(nbins), s);
        scan_i32_to_i32(bmc.p, g.bm_start.p, nbins, g.scan_tmp.p, s);
        // every (bin, macro) pair at most once: size the list by that bound
        // unless it is large, and only then read the exact count
        const int64_t bound = static_cast<int64_t>(n_macro) * nbins;
        const int64_t nbm = bound <= (int64_t(1) << 24) ? bound : read_i32(g.bm_start.p + nbins, s);
        g.bm_list.ensure(static_cast<size_t>(nbm) + 1, s);
        hipLaunchKernelGGL(k_bin_macros, dim3(nbins), dim3(kBT), 0, s, hp.nbx, g.macro_span.p, n_macro,
                           static_cast<const int32_t*>(g.bm_start.p), static_cast<int32_t*>(nullptr), g.bm_list.p);
        AHR_LAUNCHED("k_bin_macros fill");
        bmc.release(s);
    } else if (!use_macros) {
        fill_i32(g.bm_start.p, nbins + 1, 0, s);
        g.bm_list.ensure(1, s);
    }
    g.macro_cache = g.n_movable_macro == 0 ? 1 : 0;

    HintArgs a;
    a.gr = gr;
    a.pos = pos;
    a.ncols = ncols;
    a.n_inst = n_inst;
    a.n_macro = n_macro;
    a.nbins = nbins;
    a.first_mvirt = g.first_mvirt;
    a.first_bvirt = g.first_bvirt;
    a.macro_hints = use_macros;
    a.bin_hints = bin_hints;
    a.perm = g.perm.p;
    a.cell_bin = g.cell_bin.p;
    a.bin_start = g.bin_start.p;
    a.bin_cells = g.bin_cells.p;
    a.bm_start = g.bm_start.p;
    a.bm_list = g.bm_list.p;
    a.rect = g.macro_rect.p;
    a.span = g.macro_span.p;
    a.phi = g.phi.p;
    a.base_w = g.base_w.p;
    a.xpos = g.xpos.p;
    a.xbase_w = g.xbase_w.p;
    g.xhabs.ensure(static_cast<size_t>(n_inst) + 1, s);
    g.xhsg.ensure(static_cast<size_t>(n_inst) + 1, s);
    a.habs = g.xhabs.p;
    a.hsg = g.xhsg.p;
    a.prune_tau = bin_hints ? static_cast<double>(hp.prune_tau) : 0.0;
    const int wslots = (2 * gr.hx + 1) * (2 * gr.hy + 1);
    // Pruning is decided in the count pass when a window has at most 64
    // slots (one bit each); wider windows mark holes in the fill and compact.
    const bool direct_prune = a.prune_tau > 0.0 && wslots <= 64;
    if (direct_prune) g.keep_mask.ensure(static_cast<size_t>(n_inst) + 1, s);
    a.keep_mask = direct_prune ? g.keep_mask.p : nullptr;
    a.kept = nullptr;
    a.nmac = nullptr;

    // 5. per cell: macros holding it, window size; (cell, macro) pairs
    g.nmac.ensure(static_cast<size_t>(n_inst) + 1, s);
    g.nwin.ensure(static_cast<size_t>(n_inst) + 1, s);
    hipLaunchKernelGGL(k_cell_count, dim3(grid_for(n_inst, kBT)), dim3(kBT), 0, s, a, g.nmac.p, g.nwin.p,
                       static_cast<const int32_t*>(nullptr), static_cast<int32_t*>(nullptr),
                       static_cast<int32_t*>(nullptr));
    AHR_LAUNCHED("k_cell_count");
    a.nmac = g.nmac.p;
    g.pair_off.ensure(static_cast<size_t>(n_inst) + 1, s);
    g.scan_tmp.ensure(scan_tmp_elems(std::max<int64_t>(N, n_inst)), s);
    scan_i32_to_i32(g.nmac.p, g.pair_off.p, n_inst, g.scan_tmp.p, s);
    // (the netlist entry count rides along: the build sizes its arrays by a
    // bound and leaves the exact count to this read)
    int32_t tot[3];
    read_scalars({g.pair_off.p + n_inst, g.bin_start.p + nbins, g.xnet_rp.p + N}, tot, s);
    const int32_t n_pairs = tot[0];
    g.n_hint_cells = tot[1];
    g.nnz_net = tot[2];
    // pruned bin rows: tiles of kBT cells within each bin, the kept cells per
    // (tile, slot) turned into carries, and per (bin, slot) totals
    DevBuf<int32_t> tile_start, tile_carry;
    const int32_t max_tiles = direct_prune ? g.n_hint_cells / kBT + nbins : 0;
    if (direct_prune) {
        DevBuf<int32_t> ntiles;
        ntiles.ensure(static_cast<size_t>(nbins) + 1, s);
        tile_start.ensure(static_cast<size_t>(nbins) + 1, s);
        tile_carry.ensure(static_cast<size_t>(max_tiles) * wslots + 1, s);
        g.kept.ensure(static_cast<size_t>(nbins) * wslots + 1, s);
        hipLaunchKernelGGL(k_bin_tile_counts, dim3(grid_for(nbins, kBT)), dim3(kBT), 0, s, g.bin_start.p, nbins,
                           ntiles.p);
        AHR_LAUNCHED("k_bin_tile_counts");
        scan_i32_to_i32(ntiles.p, tile_start.p, nbins, g.scan_tmp.p, s);
        ntiles.release(s);
        hipLaunchKernelGGL(k_tile_keep_counts, dim3(max_tiles), dim3(kBT), 0, s, a, tile_start.p, wslots,
                           tile_carry.p);
        AHR_LAUNCHED("k_tile_keep_counts");
        hipLaunchKernelGGL(k_tile_carry, dim3(grid_for(static_cast<int64_t>(nbins) * wslots, kBT)), dim3(kBT), 0, s,
                           tile_start.p, nbins, wslots, tile_carry.p, g.kept.p);
        AHR_LAUNCHED("k_tile_carry");
        a.kept = g.kept.p;
    }
    g.pair_row.ensure(static_cast<size_t>(n_pairs) + 1, s);
    g.pair_mac.ensure(static_cast<size_t>(n_pairs) + 1, s);
    if (n_pairs) {
        hipLaunchKernelGGL(k_cell_count, dim3(grid_for(n_inst, kBT)), dim3(kBT), 0, s, a,
                           static_cast<int32_t*>(nullptr), static_cast<int32_t*>(nullptr),
                           static_cast<const int32_t*>(g.pair_off.p), g.pair_row.p, g.pair_mac.p);
        AHR_LAUNCHED("k_cell_count pairs");
    }
    // pairs grouped by macro, ascending row: the macro virtual rows
    if (use_macros) bucket_sort(g, g.pair_mac.p, n_pairs, n_macro, g.mlist, g.mstart, s, false);

    // 6. row counts and offsets (execution order)
    {
        const int32_t cb = static_cast<int32_t>(grid_for(n_inst, kBT));
        const int32_t mb = use_macros ? static_cast<int32_t>(grid_for(n_macro, kBT)) : 0;
        const int32_t bb = bin_hints ? static_cast<int32_t>(grid_for(nbins, kBT)) : 0;
        hipLaunchKernelGGL(k_hint_row_counts, dim3(cb + mb + bb), dim3(kBT), 0, s, a, n_inst, g.nmac.p, g.nwin.p,
                           n_macro, g.first_mvirt, g.mstart.p, cb, mb, g.hint_cnt.p);
        AHR_LAUNCHED("k_hint_row_counts");
    }
    // Every entry is one side of a (cell, macro) pair or of a (hint cell,
    // window bin) pair, so the entries number at most twice the pairs plus
    // twice the hint cells times the window slots: the entry array is sized
    // by that bound without waiting for the count, which the normalisation
    // reads with its own sizes.  Near the int32 limit the exact count is read.
    const int64_t bound =
        2 * (static_cast<int64_t>(n_pairs) + (bin_hints ? static_cast<int64_t>(g.n_hint_cells) * wslots : 0));
    int64_t cap = bound;
    g.nnz_hint = -1;
    if (bound + static_cast<int64_t>(g.nnz_net) >= INT32_MAX) {
        const int64_t nnz = scan_i32_checked(g.hint_cnt.p, g.xhint_rp.p, N, g.scan_tmp.p, s);
        if (nnz + static_cast<int64_t>(g.nnz_net) >= INT32_MAX)
            throw Error{AHR_EUNSUPPORTED, "graph with hints has 2^31 or more entries"};
        g.nnz_hint = static_cast<int32_t>(nnz);
        cap = nnz;
    } else {
        scan_i32_to_i32(g.hint_cnt.p, g.xhint_rp.p, N, g.scan_tmp.p, s);
    }
    g.xhint_ent.ensure(static_cast<size_t>(cap) + 1, s);

    // 7. entries: cell rows first (their weights are reused), then virtual rows
    if (bin_hints) {
        g.bin_rank.ensure(static_cast<size_t>(n_inst) + 1, s);
        g.wpre.ensure(static_cast<size_t>(nbins) * wslots + 1, s);
        if (g.n_hint_cells && !direct_prune)
            hipLaunchKernelGGL(k_bin_rank, dim3(grid_for(g.n_hint_cells, kBT)), dim3(kBT), 0, s, g.n_hint_cells,
                               g.bin_cells.p, g.bin_rank.p);
        AHR_LAUNCHED("k_bin_rank");
        hipLaunchKernelGGL(k_window_prefix, dim3(grid_for(nbins, kBT)), dim3(kBT), 0, s, a, g.wpre.p);
        AHR_LAUNCHED("k_window_prefix");
    }
    hipLaunchKernelGGL(k_cell_fill, dim3(grid_for(n_inst, kBT)), dim3(kBT), 0, s, a,
                       static_cast<const int32_t*>(g.xhint_rp.p), static_cast<const int32_t*>(g.pair_off.p),
                       static_cast<const int32_t*>(g.pair_mac.p), static_cast<const int32_t*>(g.bin_rank.p),
                       static_cast<const int32_t*>(g.wpre.p), g.xhint_ent.p);
    AHR_LAUNCHED("k_cell_fill");
    if (direct_prune) {
        hipLaunchKernelGGL(k_bin_side_fill, dim3(max_tiles), dim3(kBT), 0, s, a,
                           static_cast<const int32_t*>(tile_start.p), static_cast<const int32_t*>(tile_carry.p),
                           static_cast<const int32_t*>(g.xhint_rp.p), static_cast<const int32_t*>(g.wpre.p),
                           g.xhint_ent.p);
        AHR_LAUNCHED("k_bin_side_fill");
        tile_start.release(s);
        tile_carry.release(s);
    }
    g.habs_version = g.hint_version;
    if (use_macros && n_pairs) {
        hipLaunchKernelGGL(k_macro_fill, dim3(grid_for(n_pairs, kBT)), dim3(kBT), 0, s, n_pairs, g.first_mvirt,
                           g.mlist.p, g.mstart.p, g.pair_row.p, g.pair_mac.p, g.pair_off.p, g.xhint_rp.p,
                           g.xhint_ent.p);
        AHR_LAUNCHED("k_macro_fill");
    }
    if (a.prune_tau > 0.0 && !direct_prune && cap > 0) prune_hints(g, cap, s);
}

}  // namespace ahr
