// Area hints of one placement (Section V): bin densities D_b and
// phi_b = 2 sigmoid(mu (D_b - C)) - 1, bin-window edges
// w = -exp(-maxRatio_{i,b}) phi_b baseWeight_i, macro-footprint edges
// w = -exp(-maxRatio_{i,m}) baseWeight_i.  Which entries exist is decided in
// float32 (cell bin, footprint test) and laid out with integer counts and
// scans only, so the structure is exact and run-to-run identical; weights
// are evaluated in float64 and stored as float32, by one function per edge
// kind, so A_ij and A_ji are bit-identical.
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

__device__ __forceinline__ float w_bin(const Grid& gr, float x, float y, int b, const double* phi, double bw_i) {
    int bx = b % gr.nbx, by = b / gr.nbx;
    double xb = gr.xl + (static_cast<double>(bx) + 0.5) * gr.bw;
    double yb = gr.yl + (static_cast<double>(by) + 0.5) * gr.bh;
    double rx = fabs(static_cast<double>(x) - xb) / (gr.bw / 2);
    double ry = fabs(static_cast<double>(y) - yb) / (gr.bh / 2);
    double r = rx > ry ? rx : ry;
    return static_cast<float>(-exp(-r) * phi[b] * bw_i);
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

// Bin of every hint cell (-1 otherwise) and fixed-point cell area per bin.
__global__ void __launch_bounds__(kBT) k_cell_bins(Grid gr, const float* __restrict__ pos, int ncols, int32_t n_inst,
                                                   const uint8_t* __restrict__ flags, const float* __restrict__ size,
                                                   const int64_t* __restrict__ qdeg, int with_density,
                                                   int32_t* __restrict__ cell_bin,
                                                   unsigned long long* __restrict__ area_q) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x;
    if (i >= n_inst) return;
    uint8_t f = flags[i];
    int b = -1;
    if (is_std_movable(f)) {
        float x = pos[i * ncols], y = pos[i * ncols + 1];
        int bx = bin_coord(x, gr.xl32, gr.bw32, gr.nbx);
        int by = bin_coord(y, gr.yl32, gr.bh32, gr.nby);
        int bb = by * gr.nbx + bx;
        if (with_density) {
            double a = static_cast<double>(size[2 * i]) * static_cast<double>(size[2 * i + 1]);
            atomicAdd(&area_q[bb], static_cast<unsigned long long>(static_cast<int64_t>(__builtin_rint(a * kAreaQ))));
        }
        if (qdeg[i] > 0) b = bb;
    }
    cell_bin[i] = b;
}

// Stable bucket sort, pass 1: hint cells per (bin, tile), bin-major.
__global__ void __launch_bounds__(kWave) k_bucket_count(const int32_t* __restrict__ cell_bin, int32_t n, int nbins,
                                                        int32_t ntiles, int32_t* __restrict__ hist) {
    __shared__ int32_t h[kMaxBins];
    for (int b = threadIdx.x; b < nbins; b += kWave) h[b] = 0;
    __syncthreads();
    int64_t base = static_cast<int64_t>(blockIdx.x) * kTileCells;
    for (int t = 0; t < kTileIters; ++t) {
        int64_t i = base + t * kWave + threadIdx.x;
        if (i < n) {
            int b = cell_bin[i];
            if (b >= 0) atomicAdd(&h[b], 1);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += kWave) hist[static_cast<int64_t>(b) * ntiles + blockIdx.x] = h[b];
}

// Pass 2: place every hint cell at offset(bin, tile) + rank among the
// tile's earlier cells of the same bin (lanes in id order, tiles in order).
__global__ void __launch_bounds__(kWave) k_bucket_scatter(const int32_t* __restrict__ cell_bin, int32_t n, int nbins,
                                                          int bits, int32_t ntiles, const int32_t* __restrict__ off,
                                                          int32_t* __restrict__ out) {
    __shared__ int32_t run[kMaxBins];
    for (int b = threadIdx.x; b < nbins; b += kWave) run[b] = off[static_cast<int64_t>(b) * ntiles + blockIdx.x];
    __syncthreads();
    int l = threadIdx.x;
    uint64_t lt = l ? (~0ull >> (kWave - l)) : 0ull;
    uint64_t gt = (l == kWave - 1) ? 0ull : (~0ull << (l + 1));
    int64_t base = static_cast<int64_t>(blockIdx.x) * kTileCells;
    for (int t = 0; t < kTileIters; ++t) {
        int64_t i = base + t * kWave + l;
        int b = (i < n) ? cell_bin[i] : -1;
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

__global__ void k_bin_start(const int32_t* __restrict__ off, int nbins, int32_t ntiles, int32_t total,
                            int32_t* __restrict__ bin_start) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nbins) bin_start[b] = off[static_cast<int64_t>(b) * ntiles];
    if (b == nbins) bin_start[b] = total;
}

// Macro footprint (float32), its widened bin span, and its exact area per bin.
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
    int bx0 = bin_coord(cx - r.z, gr.xl32, gr.bw32, gr.nbx) - 1;
    int bx1 = bin_coord(cx + r.z, gr.xl32, gr.bw32, gr.nbx) + 1;
    int by0 = bin_coord(cy - r.w, gr.yl32, gr.bh32, gr.nby) - 1;
    int by1 = bin_coord(cy + r.w, gr.yl32, gr.bh32, gr.nby) + 1;
    span[k] = make_int4(bx0 < 0 ? 0 : bx0, by0 < 0 ? 0 : by0, bx1 >= gr.nbx ? gr.nbx - 1 : bx1,
                        by1 >= gr.nby ? gr.nby - 1 : by1);
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
    const int32_t* cell_bin;
    const int32_t* bin_start;
    const int32_t* bin_cells;
    const int32_t* bm_start;
    const int32_t* bm_list;
    const float4* rect;
    const int4* span;
    const double* phi;
    const double* base_w;
};

__device__ __forceinline__ void window(const Grid& gr, int b, int& x0, int& x1, int& y0, int& y1) {
    int bx = b % gr.nbx, by = b / gr.nbx;
    x0 = bx - gr.hx < 0 ? 0 : bx - gr.hx;
    x1 = bx + gr.hx >= gr.nbx ? gr.nbx - 1 : bx + gr.hx;
    y0 = by - gr.hy < 0 ? 0 : by - gr.hy;
    y1 = by + gr.hy >= gr.nby ? gr.nby - 1 : by + gr.hy;
}

// Hint entries of every cell row (pass 1: count, pass 2: write).
__global__ void __launch_bounds__(kBT) k_cell_rows(HintArgs a, int32_t* __restrict__ cnt,
                                                   const int32_t* __restrict__ rp, int2* __restrict__ ent) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x;
    if (i >= a.n_inst) return;
    int b = a.cell_bin[i];
    if (b < 0) {
        if (cnt) cnt[i] = 0;
        return;
    }
    float x = a.pos[i * a.ncols], y = a.pos[i * a.ncols + 1];
    double bwi = a.base_w[i];
    int n = 0;
    int64_t o = ent ? rp[i] : 0;
    if (a.macro_hints) {
        for (int t = a.bm_start[b]; t < a.bm_start[b + 1]; ++t) {
            int k = a.bm_list[t];
            float4 m = a.rect[k];
            if (inside(x, y, m)) {
                if (ent) ent[o + n] = make_int2(a.first_mvirt + k, f_bits(w_macro(x, y, m, bwi)));
                ++n;
            }
        }
    }
    if (a.bin_hints) {
        int x0, x1, y0, y1;
        window(a.gr, b, x0, x1, y0, y1);
        if (ent) {
            for (int by = y0; by <= y1; ++by)
                for (int bx = x0; bx <= x1; ++bx) {
                    int bb = by * a.gr.nbx + bx;
                    ent[o + n] = make_int2(a.first_bvirt + bb, f_bits(w_bin(a.gr, x, y, bb, a.phi, bwi)));
                    ++n;
                }
        } else {
            n += (x1 - x0 + 1) * (y1 - y0 + 1);
        }
    }
    if (cnt) cnt[i] = n;
}

// Macro virtual rows: one workgroup per macro walks the cells of the bins in
// its span (row-major bins, ascending cells) and keeps those inside.
__global__ void __launch_bounds__(kBT) k_macro_rows(HintArgs a, int32_t* __restrict__ cnt,
                                                    const int32_t* __restrict__ rp, int2* __restrict__ ent) {
    __shared__ int red[kBT / kWave];
    int k = blockIdx.x;
    float4 m = a.rect[k];
    int4 sp = a.span[k];
    int row = a.first_mvirt + k;
    int64_t o = ent ? rp[row] : 0;
    int carry = 0;
    for (int by = sp.y; by <= sp.w; ++by)
        for (int bx = sp.x; bx <= sp.z; ++bx) {
            int b = by * a.gr.nbx + bx;
            int s0 = a.bin_start[b], s1 = a.bin_start[b + 1];
            for (int t0 = s0; t0 < s1; t0 += kBT) {
                int t = t0 + threadIdx.x;
                int c = -1;
                bool f = false;
                float x = 0, y = 0;
                if (t < s1) {
                    c = a.bin_cells[t];
                    x = a.pos[static_cast<int64_t>(c) * a.ncols];
                    y = a.pos[static_cast<int64_t>(c) * a.ncols + 1];
                    f = inside(x, y, m);
                }
                int tot;
                int idx = block_rank<kBT>(f, red, &tot);
                if (ent && f) ent[o + carry + idx] = make_int2(c, f_bits(w_macro(x, y, m, a.base_w[c])));
                carry += tot;
            }
        }
    if (cnt && threadIdx.x == 0) cnt[row] = carry;
}

// Bin virtual rows: the cells of every bin in the window, row-major bins.
__global__ void k_bin_row_counts(HintArgs a, int32_t* __restrict__ cnt) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.nbins) return;
    int x0, x1, y0, y1;
    window(a.gr, b, x0, x1, y0, y1);
    int n = 0;
    for (int by = y0; by <= y1; ++by)
        for (int bx = x0; bx <= x1; ++bx) {
            int bb = by * a.gr.nbx + bx;
            n += a.bin_start[bb + 1] - a.bin_start[bb];
        }
    cnt[a.first_bvirt + b] = n;
}

__global__ void __launch_bounds__(kBT) k_bin_rows(HintArgs a, const int32_t* __restrict__ rp, int2* __restrict__ ent) {
    int b = blockIdx.x;
    int x0, x1, y0, y1;
    window(a.gr, b, x0, x1, y0, y1);
    int64_t o = rp[a.first_bvirt + b];
    for (int by = y0; by <= y1; ++by)
        for (int bx = x0; bx <= x1; ++bx) {
            int bb = by * a.gr.nbx + bx;
            int s0 = a.bin_start[bb], s1 = a.bin_start[bb + 1];
            for (int t = s0 + threadIdx.x; t < s1; t += kBT) {
                int c = a.bin_cells[t];
                float x = a.pos[static_cast<int64_t>(c) * a.ncols], y = a.pos[static_cast<int64_t>(c) * a.ncols + 1];
                ent[o + (t - s0)] = make_int2(c, f_bits(w_bin(a.gr, x, y, b, a.phi, a.base_w[c])));
            }
            o += s1 - s0;
        }
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

template <class T>
T read_scalar(const T* dev, hipStream_t s) {
    T v;
    AHR_HIP(hipMemcpyAsync(&v, dev, sizeof(T), hipMemcpyDeviceToHost, s));
    AHR_HIP(hipStreamSynchronize(s));
    return v;
}

int window_half(float ratio, int nb) {
    // n = max(1, floor(ratio * numBin)) in float32; the window spans +-floor(n/2)
    float p = ratio * static_cast<float>(nb);
    int n = static_cast<int>(floorf(p));
    if (n < 1) n = 1;
    return n / 2;
}

}  // namespace

void build_hints(Graph& g, const float* pos, int32_t ncols, hipStream_t s) {
    const ahr_hint_params& hp = g.hp;
    const int macro_hints = (hp.flags & AHR_MACRO_HINTS) ? 1 : 0;
    const int bin_hints = (hp.flags & AHR_BIN_HINTS) ? 1 : 0;
    const int32_t N = g.n_tot, n_inst = g.n_inst;
    g.hint_cnt.ensure(static_cast<size_t>(N) + 1, s);
    g.hint_rp.ensure(static_cast<size_t>(N) + 1, s);
    fill_i32(g.hint_cnt.p, N + 1, 0, s);
    g.hint_version++;
    g.has_hints = 1;
    if (!macro_hints && !bin_hints) {
        fill_i32(g.hint_rp.p, N + 1, 0, s);
        g.nnz_hint = 0;
        g.n_hint_cells = 0;
        g.hint_ent.ensure(1, s);
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

    // 1. cell bins and cell areas
    g.cell_bin.ensure(static_cast<size_t>(n_inst) + 1, s);
    g.bin_area_q.ensure(static_cast<size_t>(nbins) + 1, s);
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(nbins, kBT)), dim3(kBT), 0, s,
                       reinterpret_cast<unsigned long long*>(g.bin_area_q.p), static_cast<int64_t>(nbins));
    AHR_LAUNCHED("k_fill_u64");
    hipLaunchKernelGGL(k_cell_bins, dim3(grid_for(n_inst, kBT)), dim3(kBT), 0, s, gr, pos, ncols, n_inst,
                       g.nl.node_flags, g.nl.node_size, g.qdeg.p, bin_hints, g.cell_bin.p,
                       reinterpret_cast<unsigned long long*>(g.bin_area_q.p));
    AHR_LAUNCHED("k_cell_bins");

    // 2. hint cells grouped by bin, ascending ids (stable bucket sort)
    int32_t ntiles = static_cast<int32_t>((n_inst + kTileCells - 1) / kTileCells);
    int64_t hn = static_cast<int64_t>(nbins) * ntiles;
    g.i32a.ensure(static_cast<size_t>(hn) + 1, s);
    g.i32b.ensure(static_cast<size_t>(hn) + 1, s);
    hipLaunchKernelGGL(k_bucket_count, dim3(ntiles), dim3(kWave), 0, s, g.cell_bin.p, n_inst, nbins, ntiles, g.i32a.p);
    AHR_LAUNCHED("k_bucket_count");
    g.scan_tmp.ensure(scan_tmp_elems(hn), s);
    scan_i32_to_i32(g.i32a.p, g.i32b.p, hn, g.scan_tmp.p, s);
    g.n_hint_cells = read_scalar(g.i32b.p + hn, s);
    g.bin_cells.ensure(static_cast<size_t>(g.n_hint_cells) + 1, s);
    int bits = 0;
    while ((1 << bits) < nbins) ++bits;
    hipLaunchKernelGGL(k_bucket_scatter, dim3(ntiles), dim3(kWave), 0, s, g.cell_bin.p, n_inst, nbins, bits, ntiles,
                       g.i32b.p, g.bin_cells.p);
    AHR_LAUNCHED("k_bucket_scatter");
    g.bin_start.ensure(static_cast<size_t>(nbins) + 1, s);
    hipLaunchKernelGGL(k_bin_start, dim3(grid_for(nbins + 1, kBT)), dim3(kBT), 0, s, g.i32b.p, nbins, ntiles,
                       g.n_hint_cells, g.bin_start.p);
    AHR_LAUNCHED("k_bin_start");

    // 3. macros: footprints, spans, areas
    const int32_t n_macro = macro_hints || bin_hints ? g.n_macro : 0;
    g.macro_rect.ensure(static_cast<size_t>(n_macro) + 1, s);
    g.macro_span.ensure(static_cast<size_t>(n_macro) + 1, s);
    if (n_macro)
        hipLaunchKernelGGL(k_macros, dim3(grid_for(n_macro, kBT)), dim3(kBT), 0, s, gr, pos, ncols, g.macro_ids.p,
                           n_macro, g.nl.node_size, bin_hints, g.macro_rect.p, g.macro_span.p,
                           reinterpret_cast<unsigned long long*>(g.bin_area_q.p));
    AHR_LAUNCHED("k_macros");
    g.phi.ensure(static_cast<size_t>(nbins) + 1, s);
    if (bin_hints) {
        hipLaunchKernelGGL(k_phi, dim3(grid_for(nbins, kBT)), dim3(kBT), 0, s, nbins, gr.bw * gr.bh,
                           static_cast<double>(hp.bin_capacity), static_cast<double>(hp.mu),
                           reinterpret_cast<const unsigned long long*>(g.bin_area_q.p), g.phi.p);
        AHR_LAUNCHED("k_phi");
    }

    // 4. macros per bin
    g.bm_start.ensure(static_cast<size_t>(nbins) + 1, s);
    if (macro_hints && n_macro) {
        DevBuf<int32_t> bmc;
        bmc.ensure(static_cast<size_t>(nbins) + 1, s);
        hipLaunchKernelGGL(k_bin_macros, dim3(nbins), dim3(kBT), 0, s, hp.nbx, g.macro_span.p, n_macro,
                           static_cast<const int32_t*>(nullptr), bmc.p, static_cast<int32_t*>(nullptr));
        AHR_LAUNCHED("k_bin_macros count");
        scan_i32_to_i32(bmc.p, g.bm_start.p, nbins, g.scan_tmp.p, s);
        int32_t nbm = read_scalar(g.bm_start.p + nbins, s);
        g.bm_list.ensure(static_cast<size_t>(nbm) + 1, s);
        hipLaunchKernelGGL(k_bin_macros, dim3(nbins), dim3(kBT), 0, s, hp.nbx, g.macro_span.p, n_macro,
                           static_cast<const int32_t*>(g.bm_start.p), static_cast<int32_t*>(nullptr), g.bm_list.p);
        AHR_LAUNCHED("k_bin_macros fill");
        bmc.release(s);
    } else {
        fill_i32(g.bm_start.p, nbins + 1, 0, s);
        g.bm_list.ensure(1, s);
    }

    HintArgs a;
    a.gr = gr;
    a.pos = pos;
    a.ncols = ncols;
    a.n_inst = n_inst;
    a.n_macro = n_macro;
    a.nbins = nbins;
    a.first_mvirt = g.first_mvirt;
    a.first_bvirt = g.first_bvirt;
    a.macro_hints = macro_hints && n_macro > 0;
    a.bin_hints = bin_hints;
    a.cell_bin = g.cell_bin.p;
    a.bin_start = g.bin_start.p;
    a.bin_cells = g.bin_cells.p;
    a.bm_start = g.bm_start.p;
    a.bm_list = g.bm_list.p;
    a.rect = g.macro_rect.p;
    a.span = g.macro_span.p;
    a.phi = g.phi.p;
    a.base_w = g.base_w.p;

    // 5. row counts, offsets, entries
    hipLaunchKernelGGL(k_cell_rows, dim3(grid_for(n_inst, kBT)), dim3(kBT), 0, s, a, g.hint_cnt.p,
                       static_cast<const int32_t*>(nullptr), static_cast<int2*>(nullptr));
    AHR_LAUNCHED("k_cell_rows count");
    if (a.macro_hints) {
        hipLaunchKernelGGL(k_macro_rows, dim3(n_macro), dim3(kBT), 0, s, a, g.hint_cnt.p,
                           static_cast<const int32_t*>(nullptr), static_cast<int2*>(nullptr));
        AHR_LAUNCHED("k_macro_rows count");
    }
    if (bin_hints) {
        hipLaunchKernelGGL(k_bin_row_counts, dim3(grid_for(nbins, kBT)), dim3(kBT), 0, s, a, g.hint_cnt.p);
        AHR_LAUNCHED("k_bin_row_counts");
    }
    DevBuf<int64_t> rp64;
    rp64.ensure(static_cast<size_t>(N) + 1, s);
    g.scan_tmp.ensure(scan_tmp_elems(N), s);
    scan_i32_to_i64(g.hint_cnt.p, rp64.p, N, g.scan_tmp.p, s);
    int64_t nnz = read_scalar(rp64.p + N, s);
    rp64.release(s);
    if (nnz + static_cast<int64_t>(g.nnz_net) >= INT32_MAX)
        throw Error{AHR_EUNSUPPORTED, "graph with hints has 2^31 or more entries"};
    scan_i32_to_i32(g.hint_cnt.p, g.hint_rp.p, N, g.scan_tmp.p, s);
    g.nnz_hint = static_cast<int32_t>(nnz);
    g.hint_ent.ensure(static_cast<size_t>(nnz) + 1, s);
    hipLaunchKernelGGL(k_cell_rows, dim3(grid_for(n_inst, kBT)), dim3(kBT), 0, s, a, static_cast<int32_t*>(nullptr),
                       static_cast<const int32_t*>(g.hint_rp.p), g.hint_ent.p);
    AHR_LAUNCHED("k_cell_rows fill");
    if (a.macro_hints) {
        hipLaunchKernelGGL(k_macro_rows, dim3(n_macro), dim3(kBT), 0, s, a, static_cast<int32_t*>(nullptr),
                           static_cast<const int32_t*>(g.hint_rp.p), g.hint_ent.p);
        AHR_LAUNCHED("k_macro_rows fill");
    }
    if (bin_hints) {
        hipLaunchKernelGGL(k_bin_rows, dim3(nbins), dim3(kBT), 0, s, a, static_cast<const int32_t*>(g.hint_rp.p),
                           g.hint_ent.p);
        AHR_LAUNCHED("k_bin_rows");
    }
}

}  // namespace ahr
