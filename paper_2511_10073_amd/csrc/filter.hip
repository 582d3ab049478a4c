// The refinement filter (Section V, eq. "refine-filter"):
//   L = diag(nz) - S (A + sigma I) S,  S = diag(s), s_i = (d_i)^-1/2,
//   d_i = sum_j |A_ij| + sigma (absolute degree: the reading for signed
//   graphs that keeps L positive semi-definite),
//   lambda_up = max_i (L_ii + sum_j |L_ij|) (Gershgorin), T = I - L/lambda_up,
//   out = sum_b alpha_b T^{k_b} X, then fixed and virtual rows reset to X.
//
// The chain runs in scaled coordinates z = S y, where one hop is
//   z'_i = c_i z_i + (s_i^2 / lambda) sum_j A_ij z_j,
//   c_i  = 1 - (nz_i - sigma s_i^2) / lambda,
// so a hop streams the unscaled adjacency once (8 bytes per entry: column and
// float32 weight) and gathers one C-wide row of z per entry; nothing is
// rescaled when the hints change.  Isolated rows (s_i = 0) are identity
// rows and are recovered from the input at the end.
//
// Rows with up to kLongRow entries are handled by G lanes each; longer rows
// (bin and macro virtual nodes, big-net stars) are split into kChunk-entry
// chunks, one workgroup each, whose float64 partial sums a small kernel adds
// after the hop in a fixed order -- deterministic for any schedule.
#include <hip/hip_ext.h>

#include "ahr_internal.hpp"
#include "device_util.hpp"

namespace ahr {

extern int g_hop_lanes;   // lanes per short row of a hop
extern int g_hop_nt;      // stream the entries with non-temporal loads

namespace {

constexpr int kBT = 256;

// ---------------------------------------------------------------- vectors

template <int C>
struct Vec {
    float v[C];
};

template <int C>
__device__ __forceinline__ Vec<C> vload(const float* p) {
    Vec<C> r;
    if constexpr (C == 1) {
        r.v[0] = p[0];
    } else if constexpr (C == 2) {
        float2 t = *reinterpret_cast<const float2*>(p);
        r.v[0] = t.x;
        r.v[1] = t.y;
    } else {
#pragma unroll
        for (int q = 0; q < C / 4; ++q) {
            float4 t = reinterpret_cast<const float4*>(p)[q];
            r.v[4 * q] = t.x;
            r.v[4 * q + 1] = t.y;
            r.v[4 * q + 2] = t.z;
            r.v[4 * q + 3] = t.w;
        }
    }
    return r;
}

template <int C>
__device__ __forceinline__ void vstore(float* p, const Vec<C>& r) {
    if constexpr (C == 1) {
        p[0] = r.v[0];
    } else if constexpr (C == 2) {
        *reinterpret_cast<float2*>(p) = make_float2(r.v[0], r.v[1]);
    } else {
#pragma unroll
        for (int q = 0; q < C / 4; ++q)
            reinterpret_cast<float4*>(p)[q] = make_float4(r.v[4 * q], r.v[4 * q + 1], r.v[4 * q + 2], r.v[4 * q + 3]);
    }
}

// A first-hop record: a row's C signal columns, then its scale, with no
// padding (C + 1 floats, 4-byte aligned).  Padding to a power of two kept
// every record inside one cache line but made the records' footprint, which
// the first hop gathers from, nearly twice the signal's; the tight records
// cost a second line for a few of them and fewer lines in all.
template <int C>
constexpr int pack_width() {
    static_assert(C <= 4, "first-hop records hold at most 4 columns");
    return C + 1;
}

// W floats at a 4-byte aligned address (a record, or its columns).
template <int W>
struct alignas(4) Floats {
    float v[W];
};

template <int W>
__device__ __forceinline__ Floats<W> load_floats(const float* p) {
    return *reinterpret_cast<const Floats<W>*>(p);
}

// ---------------------------------------------------------------- row classes

__global__ void k_row_len(int32_t n, const int32_t* __restrict__ net_rp, const int32_t* __restrict__ hint_rp,
                          int32_t* __restrict__ is_long) {
    int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int len = (net_rp[r + 1] - net_rp[r]) + (hint_rp[r + 1] - hint_rp[r]);
    is_long[r] = len > kLongRow ? 1 : 0;
}

// Long-row flag and chunk count of every row (0 for short rows).
__global__ void k_row_chunks(int32_t n, const int32_t* __restrict__ net_rp, const int32_t* __restrict__ hint_rp,
                             int32_t* __restrict__ is_long, int32_t* __restrict__ nch) {
    int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int len = (net_rp[r + 1] - net_rp[r]) + (hint_rp[r + 1] - hint_rp[r]);
    bool lg = len > kLongRow;
    is_long[r] = lg ? 1 : 0;
    nch[r] = lg ? (len + kChunk - 1) / kChunk : 0;
}

// First chunk of each long row from the row-indexed chunk offsets; the
// entry past the last row holds the chunk total.
__global__ void k_long_chunk0(int32_t n_long, const int32_t* __restrict__ rows, const int32_t* __restrict__ cscan,
                              int32_t n_chunks, int32_t* __restrict__ chunk0) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_long) chunk0[i] = cscan[rows[i]];
    if (i == n_long) chunk0[i] = n_chunks;
}

__global__ void k_chunk_rows(int32_t n_long, const int32_t* __restrict__ chunk0, int32_t* __restrict__ chunk_row) {
    int i = blockIdx.x;
    if (i >= n_long) return;
    for (int c = chunk0[i] + threadIdx.x; c < chunk0[i + 1]; c += blockDim.x) chunk_row[c] = i;
}

struct RowRef {
    const int32_t* net_rp;
    const int2* net_ent;
    const int32_t* hint_rp;
    const int2* hint_ent;
};

// Row blocks: a short row starts a block when it is the first row, the
// first instance or auxiliary row, follows a long row, or when its combined
// entry offset (netlist + hints) or its index enters a new window of
// kRbEntries entries / kRbRows rows; it ends one when the next row starts
// one or is long.  A block so has at most kRbRows rows and fewer than
// kRbEntries + kLongRow entries.
__device__ __forceinline__ bool rb_break(int32_t r, int32_t n_inst, const int32_t* net_rp, const int32_t* hint_rp) {
    // is there a block boundary between rows r - 1 and r (both short)?
    const int64_t c1 = static_cast<int64_t>(net_rp[r]) + hint_rp[r];
    const int64_t c0 = static_cast<int64_t>(net_rp[r - 1]) + hint_rp[r - 1];
    return r == n_inst || c1 / kRbEntries != c0 / kRbEntries || r / kRbRows != (r - 1) / kRbRows;
}

__global__ void k_rb_marks(int32_t n, int32_t n_inst, const int32_t* __restrict__ net_rp,
                           const int32_t* __restrict__ hint_rp, const int32_t* __restrict__ is_long,
                           int32_t* __restrict__ start, int32_t* __restrict__ end) {
    int64_t r64 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r64 >= n) return;
    const int32_t r = static_cast<int32_t>(r64);
    int32_t st = 0, en = 0;
    if (!is_long[r]) {
        st = (r == 0 || is_long[r - 1] || rb_break(r, n_inst, net_rp, hint_rp)) ? 1 : 0;
        en = (r == n - 1 || is_long[r + 1] || rb_break(r + 1, n_inst, net_rp, hint_rp)) ? 1 : 0;
    }
    start[r] = st;
    end[r] = en;
}

__global__ void k_rb_desc(int32_t n_rb, const int32_t* __restrict__ starts, const int32_t* __restrict__ ends,
                          const int32_t* __restrict__ net_rp, const int32_t* __restrict__ hint_rp, int4* __restrict__ rb) {
    int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n_rb) return;
    const int32_t r0 = starts[k], r1 = ends[k] + 1;
    rb[2 * k] = make_int4(r0, r1, net_rp[r0], net_rp[r1]);
    rb[2 * k + 1] = make_int4(hint_rp[r0], hint_rp[r1], 0, 0);
}

__global__ void k_coef(int32_t n, const float* __restrict__ scale, const double* __restrict__ lam, double sigma,
                       float2* __restrict__ coef) {
    int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    float cr, kr;
    hop_coef(scale[r], *lam, sigma, cr, kr);
    coef[r] = make_float2(cr, kr);
}

// ---------------------------------------------------------------- degrees

// Degree d_i = qdeg_i 2^-32 + sum_j |hint_ij| + sigma, scale s_i = d_i^-1/2,
// and the signed sum of the row's hint weights (a feature of the learned
// surrogate).
// Lane t of the rows from r0 on, G lanes per row.
template <int G>
__device__ __forceinline__ void deg_short_row(int64_t t, int32_t r0, int32_t n, const RowRef& m,
                                              const int64_t* __restrict__ qdeg, double sigma,
                                              double* __restrict__ deg, float* __restrict__ scale,
                                              float* __restrict__ hsum) {
    int64_t r = r0 + t / G;
    int l = static_cast<int>(t & (G - 1));
    if (r >= n) return;
    int h0 = m.hint_rp[r], h1 = m.hint_rp[r + 1];
    int len = (m.net_rp[r + 1] - m.net_rp[r]) + (h1 - h0);
    if (len > kLongRow) return;
    double a = 0, sg = 0;
    for (int k = h0 + l; k < h1; k += G) {
        double w = static_cast<double>(bits_f(m.hint_ent[k].y));
        a += fabs(w);
        sg += w;
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        sg += __shfl_xor(sg, o);
    }
    if (l == 0) {
        double d = static_cast<double>(qdeg[r]) * 0x1p-32 + a + sigma;
        deg[r] = d;
        scale[r] = d > 0 ? static_cast<float>(1.0 / sqrt(d)) : 0.f;
        hsum[r] = static_cast<float>(sg);
    }
}

// The same for the short cell rows, from the hint sums the hint build
// formed for every cell.
__device__ __forceinline__ void deg_cell_row(int64_t r, int32_t n_inst, const RowRef& m,
                                             const int64_t* __restrict__ qdeg, const double* __restrict__ habs,
                                             const float* __restrict__ hsg, double sigma, double* __restrict__ deg,
                                             float* __restrict__ scale, float* __restrict__ hsum) {
    if (r >= n_inst) return;
    int len = (m.net_rp[r + 1] - m.net_rp[r]) + (m.hint_rp[r + 1] - m.hint_rp[r]);
    if (len > kLongRow) return;
    double d = static_cast<double>(qdeg[r]) * 0x1p-32 + habs[r] + sigma;
    deg[r] = d;
    scale[r] = d > 0 ? static_cast<float>(1.0 / sqrt(d)) : 0.f;
    hsum[r] = hsg[r];
}

// Both in one launch: the first cell_blocks workgroups take the cell rows
// below r0 (one lane each), the rest G lanes per row from r0 to n.
template <int G>
__global__ void __launch_bounds__(kBT) k_deg_rows(int32_t r0, int32_t n, int32_t cell_blocks, RowRef m,
                                                  const int64_t* __restrict__ qdeg, const double* __restrict__ habs,
                                                  const float* __restrict__ hsg, double sigma,
                                                  double* __restrict__ deg, float* __restrict__ scale,
                                                  float* __restrict__ hsum) {
    const int32_t b = static_cast<int32_t>(blockIdx.x);
    if (b < cell_blocks)
        deg_cell_row(static_cast<int64_t>(b) * kBT + threadIdx.x, r0, m, qdeg, habs, hsg, sigma, deg, scale, hsum);
    else
        deg_short_row<G>(static_cast<int64_t>(b - cell_blocks) * kBT + threadIdx.x, r0, n, m, qdeg, sigma, deg,
                         scale, hsum);
}

__device__ __forceinline__ void chunk_range(int c, const int32_t* long_rows, const int32_t* chunk_row,
                                            const int32_t* chunk0, const RowRef& m, int& r, int& li, int& k0, int& k1,
                                            int& n0, int& ln, int& h0) {
    li = chunk_row[c];
    r = long_rows[li];
    n0 = m.net_rp[r];
    ln = m.net_rp[r + 1] - n0;
    h0 = m.hint_rp[r];
    int len = ln + (m.hint_rp[r + 1] - h0);
    k0 = (c - chunk0[li]) * kChunk;
    k1 = k0 + kChunk < len ? k0 + kChunk : len;
}

__global__ void __launch_bounds__(kBT) k_chunk_absdeg(RowRef m, const int32_t* __restrict__ long_rows,
                                                      const int32_t* __restrict__ chunk_row,
                                                      const int32_t* __restrict__ chunk0, double* __restrict__ partial) {
    __shared__ double red[kBT / kWave];
    int r, li, k0, k1, n0, ln, h0;
    chunk_range(blockIdx.x, long_rows, chunk_row, chunk0, m, r, li, k0, k1, n0, ln, h0);
    // the lane's entries k0 + t + u kBT (ascending), all loaded at once: a
    // net entry or a slot past the chunk reads the row's first hint slot (the
    // hint array holds one more than its count) and adds nothing
    constexpr int U = kChunk / kBT;
    float wv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int k = k0 + static_cast<int>(threadIdx.x) + u * kBT;
        const int kh = k < k1 && k >= ln ? k - ln : 0;
        wv[u] = bits_f(m.hint_ent[h0 + kh].y);
    }
    double a = 0, sg = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int k = k0 + static_cast<int>(threadIdx.x) + u * kBT;
        if (k < k1 && k >= ln) {
            const double w = static_cast<double>(wv[u]);
            a += fabs(w);
            sg += w;
        }
    }
    a = block_sum_f64<kBT>(a, red);
    sg = block_sum_f64<kBT>(sg, red);
    if (threadIdx.x == 0) {
        partial[static_cast<int64_t>(blockIdx.x) * 8] = a;
        partial[static_cast<int64_t>(blockIdx.x) * 8 + 1] = sg;
    }
}

__global__ void k_long_deg_final(int32_t n_long, const int32_t* __restrict__ long_rows,
                                 const int32_t* __restrict__ chunk0, const double* __restrict__ partial,
                                 const int64_t* __restrict__ qdeg, double sigma, double* __restrict__ deg,
                                 float* __restrict__ scale, float* __restrict__ hsum) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_long) return;
    int r = long_rows[i];
    double a = 0, sg = 0;
    for (int c = chunk0[i]; c < chunk0[i + 1]; ++c) {
        a += partial[static_cast<int64_t>(c) * 8];
        sg += partial[static_cast<int64_t>(c) * 8 + 1];
    }
    double d = static_cast<double>(qdeg[r]) * 0x1p-32 + a + sigma;
    deg[r] = d;
    scale[r] = d > 0 ? static_cast<float>(1.0 / sqrt(d)) : 0.f;
    hsum[r] = static_cast<float>(sg);
}

// ---------------------------------------------------------------- Gershgorin

__device__ __forceinline__ double diag_abs(float s, double d, double sigma) {
    double nz = d > 0 ? 1.0 : 0.0;
    double sd = static_cast<double>(s);
    return fabs(nz - sigma * sd * sd);
}

__device__ __forceinline__ void atomic_max_nonneg(double* p, double v) {
    atomicMax(reinterpret_cast<unsigned long long*>(p), static_cast<unsigned long long>(__double_as_longlong(v)));
}

// Grid-stride over rows (G lanes per row, kGU entries per lane per batch);
// each workgroup keeps its running maximum and issues one atomic at the end
// (the maximum is order-independent).
constexpr int kGershGrid = 2048;
constexpr int kGU = 4;

template <int G>
__global__ void __launch_bounds__(kBT) k_gersh_short(int32_t n, RowRef m, const double* __restrict__ deg,
                                                     const float* __restrict__ scale, double sigma,
                                                     double* __restrict__ lam) {
    __shared__ double red[kBT / kWave];
    const int l = threadIdx.x & (G - 1);
    const int64_t stride = static_cast<int64_t>(kGershGrid) * (kBT / G);
    double best = 0;
    for (int64_t r = (static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x) / G; r < n; r += stride) {
        int n0 = m.net_rp[r], n1 = m.net_rp[r + 1], h0 = m.hint_rp[r], h1 = m.hint_rp[r + 1];
        if ((n1 - n0) + (h1 - h0) > kLongRow) continue;          // group-uniform
        const int ln = n1 - n0, len = ln + (h1 - h0);
        double a = 0;
        for (int k0 = l; k0 < len; k0 += G * kGU) {
            int2 e[kGU];
            float sc[kGU];
#pragma unroll
            for (int u = 0; u < kGU; ++u) {
                int k = k0 + u * G;
                int kc = k < len ? k : len - 1;
                e[u] = kc < ln ? m.net_ent[n0 + kc] : m.hint_ent[h0 + kc - ln];
                if (k >= len) e[u].y = 0;
            }
#pragma unroll
            for (int u = 0; u < kGU; ++u) sc[u] = scale[e[u].x];
#pragma unroll
            for (int u = 0; u < kGU; ++u) a += fabs(static_cast<double>(bits_f(e[u].y))) * static_cast<double>(sc[u]);
        }
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) a += __shfl_xor(a, o);
        if (l == 0) {
            float s = scale[r];
            double rr = diag_abs(s, deg[r], sigma) + static_cast<double>(s) * a;
            best = rr > best ? rr : best;
        }
    }
    best = wave_max(best);
    __syncthreads();
    if (lane_id() == 0) red[wave_id()] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = red[0];
        for (int w = 1; w < kBT / kWave; ++w) b = red[w] > b ? red[w] : b;
        atomic_max_nonneg(lam, b);
    }
}

__global__ void __launch_bounds__(kBT) k_chunk_gersh(RowRef m, const int32_t* __restrict__ long_rows,
                                                     const int32_t* __restrict__ chunk_row,
                                                     const int32_t* __restrict__ chunk0, const float* __restrict__ scale,
                                                     double* __restrict__ partial) {
    __shared__ double red[kBT / kWave];
    int r, li, k0, k1, n0, ln, h0;
    chunk_range(blockIdx.x, long_rows, chunk_row, chunk0, m, r, li, k0, k1, n0, ln, h0);
    double a = 0;
    for (int k = k0 + threadIdx.x; k < k1; k += kBT) {
        int2 e = k < ln ? m.net_ent[n0 + k] : m.hint_ent[h0 + k - ln];
        a += fabs(static_cast<double>(bits_f(e.y))) * static_cast<double>(scale[e.x]);
    }
    a = block_sum_f64<kBT>(a, red);
    if (threadIdx.x == 0) partial[static_cast<int64_t>(blockIdx.x) * 8] = a;
}

__global__ void k_long_gersh_final(int32_t n_long, const int32_t* __restrict__ long_rows,
                                   const int32_t* __restrict__ chunk0, const double* __restrict__ partial,
                                   const double* __restrict__ deg, const float* __restrict__ scale, double sigma,
                                   double* __restrict__ lam) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_long) return;
    int r = long_rows[i];
    double a = 0;
    for (int c = chunk0[i]; c < chunk0[i + 1]; ++c) a += partial[static_cast<int64_t>(c) * 8];
    float s = scale[r];
    atomic_max_nonneg(lam, diag_abs(s, deg[r], sigma) + static_cast<double>(s) * a);
}

__global__ void k_set_f64(double* p, double v) { *p = v; }

// ---------------------------------------------------------------- signal

// Every load unconditional and the macro-pin offset selected, so that
// callers can have several pins in flight.
template <int C>
__device__ __forceinline__ Vec<C> pin_value(const ExpandArgs& a, int p) {
    int v = a.pin_node[p];
    Vec<C> x = vload<C>(a.in + static_cast<int64_t>(v) * C);
    const bool mp = a.pin_node_x[p] >= a.n_inst;
    const float dx = a.pin_off[2 * p], dy = a.pin_off[2 * p + 1];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const float t = x.v[c] + ((c & 1) ? dy : dx);
        x.v[c] = mp ? t : x.v[c];
    }
    return x;
}

template <int C>
__device__ __forceinline__ void put_z(const ExpandArgs& a, int r, Vec<C> x, float s) {
    const int64_t row = r < a.n_inst ? static_cast<int64_t>(a.row_inst0) + r
                                     : static_cast<int64_t>(a.row_aux0) + (r - a.n_inst);
    Vec<C> z, t;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        z.v[c] = s * x.v[c];
        t.v[c] = z.v[c] * a.alpha0;
    }
    if constexpr (C <= 4) {
        if (a.zpk) {
            constexpr int W = pack_width<C>();
            Floats<W> rec;
#pragma unroll
            for (int c = 0; c < C; ++c) rec.v[c] = z.v[c];
            rec.v[C] = s;
            *reinterpret_cast<Floats<W>*>(a.zpk + row * W) = rec;
            if (a.band0) vstore<C>(a.acc + row * C, t);
            return;
        }
    }
    if (a.ct == C) {
        vstore<C>(a.z0 + row * C, z);
        if (a.band0) vstore<C>(a.acc + row * C, t);
        return;
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int64_t i = (c / a.ct) * a.tile_stride + row * a.ct + (c % a.ct);
        a.z0[i] = z.v[c];
        if (a.band0) a.acc[i] = t.v[c];
    }
}


// One row of the extended graph (execution row r).  Stars with more than
// kStarInline pins are left to expand_bigstar.
template <int C>
__device__ __forceinline__ void expand_row(const ExpandArgs& a, int r) {
    const float sc = a.scale[r];
    Vec<C> x;
    if (r < a.n_inst) {
        x = vload<C>(a.in + static_cast<int64_t>(a.perm[r]) * C);
    } else if (r < a.first_star) {
        // the macro's position plus the pin offset
        const int4 m = a.xmpin[r - a.first_mpin];
        x = vload<C>(a.in + static_cast<int64_t>(m.x) * C);
        const float dx = __int_as_float(m.y), dy = __int_as_float(m.z);
#pragma unroll
        for (int c = 0; c < C; ++c) x.v[c] += (c & 1) ? dy : dx;
    } else if (r < a.first_mvirt) {
        int e = a.xstar_net[r - a.first_star];
        int p0 = a.net_ptr[e], p1 = a.net_ptr[e + 1];
        if (p1 - p0 > kStarInline) return;
        double acc[C];
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = 0;
        for (int p = p0; p < p1; ++p) {
            Vec<C> v = pin_value<C>(a, p);
#pragma unroll
            for (int c = 0; c < C; ++c) acc[c] += v.v[c];
        }
#pragma unroll
        for (int c = 0; c < C; ++c) x.v[c] = static_cast<float>(acc[c] / (p1 - p0));
    } else if (r < a.first_bvirt) {
        x = vload<C>(a.in + static_cast<int64_t>(a.macro_ids[r - a.first_mvirt]) * C);
    } else {
        int b = r - a.first_bvirt;
        float cx = static_cast<float>(a.xl + (static_cast<double>(b % a.nbx) + 0.5) * a.bw);
        float cy = static_cast<float>(a.yl + (static_cast<double>(b / a.nbx) + 0.5) * a.bh);
#pragma unroll
        for (int c = 0; c < C; ++c) x.v[c] = (c & 1) ? cy : cx;
    }
    put_z<C>(a, r, x, sc);
}

// Mean over the pins of star k (kStarInline < pins <= kStarMid): G lanes
// (a G-aligned group) stride the pins in float64, B pins per lane in
// flight, fixed butterfly reduction.
template <int C, int G>
__device__ __forceinline__ void expand_star(const ExpandArgs& a, int k) {
    const int e = a.star_net[k];
    const int p0 = a.net_ptr[e], p1 = a.net_ptr[e + 1];
    const int deg = p1 - p0;
    if (deg <= kStarInline || deg > kStarMid) return;   // group-uniform
    const int l = threadIdx.x & (G - 1);
    double acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0;
    constexpr int B = 8;
    for (int p = p0 + l; p < p1; p += B * G) {
        Vec<C> v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) v[u] = pin_value<C>(a, p + u * G < p1 ? p + u * G : p1 - 1);   // clamped
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (p + u * G < p1) {
#pragma unroll
                for (int c = 0; c < C; ++c) acc[c] += v[u].v[c];
            }
    }
    Vec<C> x;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        double t = acc[c];
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) t += __shfl_xor(t, o);
        x.v[c] = static_cast<float>(t / deg);
    }
    if (l == 0) {
        const int r = a.iperm[a.first_star + k];
        put_z<C>(a, r, x, a.scale[r]);
    }
}

// Mean over the pins of a big star (more than kStarMid pins): the whole
// workgroup strides the pins in float64, B pins per lane in flight, then a
// fixed-order block reduction.
template <int C>
__device__ __forceinline__ void expand_big_star(const ExpandArgs& a, int k) {
    __shared__ double red[kBT / kWave];
    const int e = a.star_net[k];
    const int p0 = a.net_ptr[e], p1 = a.net_ptr[e + 1];
    double acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0;
    constexpr int B = 8;
    for (int p = p0 + static_cast<int>(threadIdx.x); p < p1; p += B * kBT) {
        Vec<C> v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) v[u] = pin_value<C>(a, p + u * kBT < p1 ? p + u * kBT : p1 - 1);   // clamped
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (p + u * kBT < p1) {
#pragma unroll
                for (int c = 0; c < C; ++c) acc[c] += v[u].v[c];
            }
    }
    Vec<C> x;
#pragma unroll
    for (int c = 0; c < C; ++c) x.v[c] = static_cast<float>(block_sum_f64<kBT>(acc[c], red) / (p1 - p0));
    if (threadIdx.x == 0) {
        const int r = a.iperm[a.first_star + k];
        put_z<C>(a, r, x, a.scale[r]);
    }
}

// The whole expansion in one launch, its three parts side by side (they
// write disjoint rows): first one workgroup per big star, then G lanes per
// mid-size star, then one lane per row.
template <int C, int G>
__global__ void __launch_bounds__(kBT) k_expand_all(ExpandArgs a, int32_t n_star, const int32_t* __restrict__ big,
                                                    int32_t nbig, int32_t bstar) {
    const int32_t b = static_cast<int32_t>(blockIdx.x);
    if (b < nbig) {
        expand_big_star<C>(a, big[b]);
    } else if (b < nbig + bstar) {
        const int64_t k = (static_cast<int64_t>(b - nbig) * kBT + threadIdx.x) / G;
        if (k < n_star) expand_star<C, G>(a, static_cast<int>(k));
    } else {
        const int64_t r = static_cast<int64_t>(b - nbig - bstar) * kBT + threadIdx.x;
        if (r < a.n_tot) expand_row<C>(a, static_cast<int>(r));
    }
}

// Graph of workgroup b in a batched launch: the last g with first[g] <= b.
__device__ __forceinline__ int owner_of(const int32_t* __restrict__ first, int32_t ng, int32_t b) {
    int lo = 0, hi = ng;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (first[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <int C>
__global__ void __launch_bounds__(kBT) k_expand_batch(const ExpandArgs* __restrict__ d, const int32_t* __restrict__ blk0,
                                                      int32_t ng, const float* __restrict__ in) {
    const int g = owner_of(blk0, ng, blockIdx.x);
    ExpandArgs a = d[g];
    a.in = in + a.in_off;
    int64_t r = static_cast<int64_t>(blockIdx.x - blk0[g]) * kBT + threadIdx.x;
    if (r < a.n_tot) expand_row<C>(a, static_cast<int>(r));
}

// G lanes per star of the batch: group w of the launch is star
// w - sfirst[g] of member g (sfirst: first star of each member, prefix sums).
template <int C, int G>
__global__ void __launch_bounds__(kBT) k_expand_star_batch(const ExpandArgs* __restrict__ d,
                                                           const int32_t* __restrict__ sfirst, int32_t ng,
                                                           int32_t n_star, const float* __restrict__ in) {
    const int64_t w = (static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x) / G;
    if (w >= n_star) return;
    const int g = owner_of(sfirst, ng, static_cast<int32_t>(w));
    ExpandArgs a = d[g];
    a.in = in + a.in_off;
    expand_star<C, G>(a, static_cast<int>(w) - sfirst[g]);
}

// One workgroup per big star of the batch (batch star indices).
template <int C>
__global__ void __launch_bounds__(kBT) k_expand_big_star_batch(const ExpandArgs* __restrict__ d,
                                                               const int32_t* __restrict__ sfirst, int32_t ng,
                                                               const int32_t* __restrict__ big,
                                                               const float* __restrict__ in) {
    const int w = big[blockIdx.x];
    const int g = owner_of(sfirst, ng, w);
    ExpandArgs a = d[g];
    a.in = in + a.in_off;
    expand_big_star<C>(a, w - sfirst[g]);
}

// ---------------------------------------------------------------- hop

struct HopArgs {
    RowRef m;
    const float* scale;
    const float2* coef;       // per-row hop coefficients, or null: from *lam
    const double* lam;
    double sigma;
    const float* zin;
    float* zout;
    float* acc;
    const float* gin;         // caller's input [n_inst][C], instance order
    float* out;               // caller's output [n_inst][C], instance order
    const uint8_t* flags;
    const int32_t* perm;      // execution row -> instance
    int32_t n_rows;           // rows of the short path
    int32_t n_chunk_blocks;   // chunk workgroups of this hop (placed first)
    const int32_t* long_rows;
    const int32_t* chunk_row;
    const int32_t* chunk0;
    double* partial;
    const int4* rb;           // row blocks (two int4 each)
    int32_t n_rb;             // row blocks of this hop (placed after the chunk workgroups)
    int band;                 // 0: none, 1: acc = alpha z', 2: acc += alpha z'
    float alpha;
    int last;
    float alpha_sum;
    int64_t tile_stride;      // elements between column tiles of zin / zout / acc
    int32_t ldo;              // columns of the caller's in / out rows
    int32_t col0;             // first caller column of this launch's tile (set per workgroup)
};

// Column tile blockIdx.y of a launch: C columns starting at col0 = y C;
// the signal buffers hold one [rows][C] block per tile.
template <int C>
__device__ __forceinline__ HopArgs tile_args(const HopArgs& a0) {
    HopArgs a = a0;
    const int64_t t = blockIdx.y;
    a.zin += t * a.tile_stride;
    a.zout += t * a.tile_stride;
    a.acc += t * a.tile_stride;
    a.col0 = static_cast<int32_t>(t) * C;
    a.partial += t * C;
    return a;
}

// Operands of a row's epilogue, loaded before the row's gathers so their
// latency overlaps them.
template <int C>
struct RowOps {
    Vec<C> z, acc;
    float s;
    float2 k;        // (cr, kr) when the launch carries per-row coefficients
    int inst;        // instance of the row (last hop)
    uint8_t flag;
};

template <int C>
__device__ __forceinline__ RowOps<C> row_ops(const HopArgs& a, int r) {
    RowOps<C> o;
    int64_t off = static_cast<int64_t>(r) * C;
    o.s = a.scale[r];
    if (a.coef) o.k = a.coef[r];
    o.z = vload<C>(a.zin + off);
    if (a.band == 2) o.acc = vload<C>(a.acc + off);
    o.inst = a.last ? a.perm[r] : r;
    o.flag = a.last ? a.flags[o.inst] : 0;
    return o;
}

template <int C>
__device__ __forceinline__ void epilogue(const HopArgs& a, int r, const RowOps<C>& o, const Vec<C>& sum) {
    const int64_t off = static_cast<int64_t>(r) * C;
    const int64_t oc = static_cast<int64_t>(o.inst) * a.ldo + a.col0;   // caller row of the output (last hop)
    if (a.last && (o.flag & AHR_NODE_FIXED)) {
        vstore<C>(a.out + oc, vload<C>(a.gin + oc));
        return;
    }
    const float s = o.s;
    float cr, kr;
    if (a.coef) {
        cr = o.k.x;
        kr = o.k.y;
    } else {
        hop_coef(s, *a.lam, a.sigma, cr, kr);
    }
    Vec<C> zn;
#pragma unroll
    for (int c = 0; c < C; ++c) zn.v[c] = cr * o.z.v[c] + kr * sum.v[c];
    if (a.last) {
        Vec<C> tot;
#pragma unroll
        for (int c = 0; c < C; ++c) tot.v[c] = (a.band == 2 ? o.acc.v[c] : 0.f) + a.alpha * zn.v[c];
        Vec<C> y;
        if (s > 0) {
#pragma unroll
            for (int c = 0; c < C; ++c) y.v[c] = tot.v[c] / s;
        } else {
            Vec<C> x = vload<C>(a.gin + oc);
#pragma unroll
            for (int c = 0; c < C; ++c) y.v[c] = a.alpha_sum * x.v[c];
        }
        vstore<C>(a.out + oc, y);
        return;
    }
    vstore<C>(a.zout + off, zn);
    if (a.band) {
        Vec<C> t;
#pragma unroll
        for (int c = 0; c < C; ++c) t.v[c] = (a.band == 2 ? o.acc.v[c] : 0.f) + a.alpha * zn.v[c];
        vstore<C>(a.acc + off, t);
    }
}

// Entry k of row r's concatenated (netlist, hints) list; k is clamped into
// the row by the caller.  The entries are streamed once per hop, so they
// are loaded non-temporally to leave the L2 to the gathered signal rows.
template <bool NT>
__device__ __forceinline__ int2 row_entry(const RowRef& m, int n0, int ln, int h0, int k) {
    const int2* p = k < ln ? m.net_ent + n0 + k : m.hint_ent + h0 + k - ln;
    if constexpr (NT) {
        long long v = __builtin_nontemporal_load(reinterpret_cast<const long long*>(p));
        return make_int2(static_cast<int>(v & 0xffffffffll), static_cast<int>(v >> 32));
    } else {
        return *p;
    }
}

// Sum of U entries per lane: all entry loads issue before any gather and all
// gathers before any use, so each lane keeps 2U requests in flight.
template <int C, int U, class Acc, bool NT>
__device__ __forceinline__ void gather_batch(const HopArgs& a, int n0, int ln, int h0, int len, int k0, int step,
                                             Acc* acc) {
    int2 e[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        int k = k0 + u * step;
        int kc = k < len ? k : len - 1;
        e[u] = row_entry<NT>(a.m, n0, ln, h0, kc);
        if (k >= len) e[u].y = 0;                 // weight 0 for the clamped duplicates
    }
    Vec<C> v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = vload<C>(a.zin + static_cast<int64_t>(e[u].x) * C);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        float w = bits_f(e[u].y);
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] += static_cast<Acc>(w) * static_cast<Acc>(v[u].v[c]);
    }
}

// One chunk of a long row: the workgroup's float64 partial sum goes to
// partial[chunk]; k_hop_long adds a row's partials after the launch ends (no
// device-scope fence inside the hop: on this chip that is an L2 write-back).
template <int C, bool NT>
__device__ __forceinline__ void hop_chunk(const HopArgs& a) {   // a: tile-adjusted
    __shared__ double red[kBT / kWave];
    int r, li, k0, k1, n0, ln, h0;
    chunk_range(blockIdx.x, a.long_rows, a.chunk_row, a.chunk0, a.m, r, li, k0, k1, n0, ln, h0);
    constexpr int U = kChunk / kBT;
    double acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0;
    gather_batch<C, U, double, NT>(a, n0, ln, h0, k1, k0 + threadIdx.x, kBT, acc);
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = block_sum_f64<kBT>(acc[c], red);
    if (threadIdx.x == 0) {
        double* part = a.partial + static_cast<int64_t>(blockIdx.x) * 8;
#pragma unroll
        for (int c = 0; c < C; ++c) part[c] = acc[c];
    }
}

// Long rows after a hop: one wave per row adds its chunk partials (fixed
// order: lanes stride the chunks, then a fixed butterfly) and applies the
// row epilogue.
template <int C>
__global__ void __launch_bounds__(kBT) k_hop_long(HopArgs a0, int32_t n_long_rows) {
    const HopArgs a = tile_args<C>(a0);
    const int64_t li = (static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x) / kWave;
    if (li >= n_long_rows) return;
    const int r = a.long_rows[li];
    const int c0 = a.chunk0[li], c1 = a.chunk0[li + 1];
    const int l = lane_id();
    RowOps<C> ops;
    if (l == 0) ops = row_ops<C>(a, r);
    double tot[C];
#pragma unroll
    for (int c = 0; c < C; ++c) tot[c] = 0;
    for (int q = c0 + l; q < c1; q += kWave) {
#pragma unroll
        for (int c = 0; c < C; ++c) tot[c] += a.partial[static_cast<int64_t>(q) * 8 + c];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) tot[c] = wave_sum(tot[c]);
    if (l != 0) return;
    Vec<C> sum;
#pragma unroll
    for (int c = 0; c < C; ++c) sum.v[c] = static_cast<float>(tot[c]);
    epilogue<C>(a, r, ops, sum);
}

// Workgroups of the short-row part are renumbered so that each XCD (blocks
// are dealt round-robin over the 8 XCDs) takes one contiguous range of rows:
// rows are in spatial order, so their gathers then share that XCD's L2.
constexpr int kXcds = 8;

// b in [0, nb), nb a multiple of kXcds: a bijection onto [0, nb) that gives
// XCD x (blocks b with b % kXcds == x) the tiles [x nb/8, (x+1) nb/8).
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb) {
    int64_t per = nb / kXcds;
    return (b % kXcds) * per + b / kXcds;
}

template <int C, int G, int U, bool NT>
__global__ void __launch_bounds__(kBT) k_hop(HopArgs a0) {
    const HopArgs a = tile_args<C>(a0);
    if (static_cast<int>(blockIdx.x) < a.n_chunk_blocks) {
        hop_chunk<C, NT>(a);
        return;
    }
    const int64_t nb = static_cast<int64_t>(gridDim.x) - a.n_chunk_blocks;     // a multiple of kXcds
    const int64_t tile = xcd_tile(static_cast<int64_t>(blockIdx.x) - a.n_chunk_blocks, nb);
    const int64_t r64 = (tile * kBT + threadIdx.x) / G;
    const int l = static_cast<int>(threadIdx.x & (G - 1));
    if (r64 >= a.n_rows) return;
    const int r = static_cast<int>(r64);
    const int n0 = a.m.net_rp[r], ln = a.m.net_rp[r + 1] - n0;
    const int h0 = a.m.hint_rp[r], lh = a.m.hint_rp[r + 1] - h0;
    const int len = ln + lh;
    if (len > kLongRow) return;
    RowOps<C> ops;
    if (l == 0) ops = row_ops<C>(a, r);
    float acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.f;
    for (int k0 = l; k0 < len; k0 += G * U) gather_batch<C, U, float, NT>(a, n0, ln, h0, len, k0, G, acc);
    Vec<C> sum;
#pragma unroll
    for (int c = 0; c < C; ++c) sum.v[c] = acc[c];
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
#pragma unroll
        for (int c = 0; c < C; ++c) sum.v[c] += __shfl_xor(sum.v[c], o);
    }
    if (l == 0) epilogue<C>(a, r, ops, sum);
}

// Row-block form of the hop: one workgroup per block of consecutive short
// rows.  Its entries are two contiguous ranges (netlist, hints), streamed
// with coalesced loads, kRbUnroll per thread in flight, each gathering its
// neighbour's C values; the weighted products go to LDS, and one thread per
// row adds its row's products in entry order (netlist, then hints) and
// applies the epilogue.
constexpr int kRbCap = kRbEntries + kLongRow;
constexpr int kRbUnroll = (kRbCap + kBT - 1) / kBT;

template <int C, bool NT>
__device__ __forceinline__ void hop_row_block(const HopArgs& a, int blk) {
    __shared__ __align__(16) float prod[kRbCap * C];
    __shared__ int32_t nrp[kRbRows + 1], hrp[kRbRows + 1];   // row starts in prod; [nr] = the block's end
    const int4 d0 = a.rb[2 * blk], d1 = a.rb[2 * blk + 1];
    const int r0 = d0.x, nr = d0.y - d0.x;
    const int net_lo = d0.z, en = d0.w - d0.z;
    const int hint_lo = d1.x, e = en + (d1.y - d1.x);
    const int t = threadIdx.x;
    // Every load unconditional, so that all are in flight together (a load
    // under a branch is waited for where the branch joins): loads past the
    // block's end read its last entry, and an empty block reads the first
    // netlist entry (both entry arrays hold one more than their count) and
    // then uses column 0.  The address is picked with masks, not a select the
    // compiler may turn into a branch.
    int2 ent[kRbUnroll];
    const int elast = e > 0 ? e - 1 : 0;
    const uint64_t live = e > 0 ? ~0ull : 0ull;
    const uint64_t nbase = reinterpret_cast<uint64_t>(a.m.net_ent) + static_cast<uint64_t>(net_lo) * sizeof(int2);
    const uint64_t hbase = reinterpret_cast<uint64_t>(a.m.hint_ent) +
                           (static_cast<uint64_t>(hint_lo) - static_cast<uint64_t>(en)) * sizeof(int2);
#pragma unroll
    for (int u = 0; u < kRbUnroll; ++u) {
        const int k = t + u * kBT < e ? t + u * kBT : elast;
        const uint64_t onnet = (k < en ? ~0ull : 0ull) | ~live;
        const uint64_t at = ((nbase + static_cast<uint64_t>(k) * sizeof(int2)) & onnet & live) |
                            (reinterpret_cast<uint64_t>(a.m.net_ent) & ~live) |
                            ((hbase + static_cast<uint64_t>(k) * sizeof(int2)) & ~onnet);
        const GlobalPtr<long long> p = reinterpret_cast<GlobalPtr<long long>>(at);
        long long v;
        if constexpr (NT) v = __builtin_nontemporal_load(p);
        else v = *p;
        ent[u] = make_int2(static_cast<int>(v & 0xffffffffll) & static_cast<int>(live), static_cast<int>(v >> 32));
    }
    RowOps<C> ops;
    if (t < nr) ops = row_ops<C>(a, r0 + t);
    if (t < nr) {
        nrp[t] = a.m.net_rp[r0 + t] - net_lo;
        hrp[t] = a.m.hint_rp[r0 + t] - hint_lo + en;
    }
    if (t == 0) {              // a block may have kRbRows = blockDim.x rows: its end comes from the descriptor
        nrp[nr] = en;
        hrp[nr] = e;
    }
    Vec<C> v[kRbUnroll];
#pragma unroll
    for (int u = 0; u < kRbUnroll; ++u) v[u] = vload<C>(a.zin + static_cast<int64_t>(ent[u].x) * C);
#pragma unroll
    for (int u = 0; u < kRbUnroll; ++u) {
        const int k = t + u * kBT;
        if (k < e) {
            const float w = bits_f(ent[u].y);
            Vec<C> q;
#pragma unroll
            for (int c = 0; c < C; ++c) q.v[c] = w * v[u].v[c];
            vstore<C>(prod + k * C, q);
        }
    }
    __syncthreads();
    if (t >= nr) return;
    Vec<C> sum;
#pragma unroll
    for (int c = 0; c < C; ++c) sum.v[c] = 0.f;
    for (int k = nrp[t]; k < nrp[t + 1]; ++k) {
        Vec<C> q = vload<C>(prod + k * C);
#pragma unroll
        for (int c = 0; c < C; ++c) sum.v[c] += q.v[c];
    }
    for (int k = hrp[t]; k < hrp[t + 1]; ++k) {
        Vec<C> q = vload<C>(prod + k * C);
#pragma unroll
        for (int c = 0; c < C; ++c) sum.v[c] += q.v[c];
    }
    epilogue<C>(a, r0 + t, ops, sum);
}

template <int C, bool NT>
__global__ void __launch_bounds__(kBT) k_hop_rb(HopArgs a0) {
    const HopArgs a = tile_args<C>(a0);
    if (static_cast<int>(blockIdx.x) < a.n_chunk_blocks) {
        hop_chunk<C, NT>(a);
        return;
    }
    const int64_t nb = static_cast<int64_t>(gridDim.x) - a.n_chunk_blocks;     // a multiple of kXcds
    const int64_t blk = xcd_tile(static_cast<int64_t>(blockIdx.x) - a.n_chunk_blocks, nb);
    if (blk >= a.n_rb) return;
    hop_row_block<C, NT>(a, static_cast<int>(blk));
}

// ------------------------------------------------ first hop with lambda_up
//
// When lambda_up is the Gershgorin bound and not yet known, the first hop
// also forms every row's Gershgorin sum sum_j |A_ij| s_j while it streams
// the entries, so the bound costs no pass of its own.  The expansion writes
// each row's z and s side by side in one record, so that one gather (nearly
// always one cache line) serves both.  The hop's epilogue needs lambda_up, so the rows' neighbour sums are
// stored unscaled in zout and the epilogue runs after the bound is reduced
// (k_hop1_epi).  Entry order, clamping and sums are those of k_hop and of
// k_gersh_short / k_chunk_gersh, so the results are the same bits.

// z_j and s_j of a first-hop record.
template <int C>
__device__ __forceinline__ void load_record(const float* zpk, int j, Vec<C>& z, float& sc) {
    constexpr int W = pack_width<C>();
    const Floats<W> r = load_floats<W>(zpk + static_cast<int64_t>(j) * W);
#pragma unroll
    for (int c = 0; c < C; ++c) z.v[c] = r.v[c];
    sc = r.v[C];
}

template <int C, int U>
__device__ __forceinline__ void gather_batch_gersh(const HopArgs& a, const float* zpk, int n0, int ln, int h0, int len,
                                                   int k0, int step, float* acc, double& ag) {
    int2 e[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        int k = k0 + u * step;
        int kc = k < len ? k : len - 1;
        e[u] = row_entry<false>(a.m, n0, ln, h0, kc);
        if (k >= len) e[u].y = 0;
    }
    Vec<C> v[U];
    float sc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) load_record<C>(zpk, e[u].x, v[u], sc[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        float w = bits_f(e[u].y);
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] += w * v[u].v[c];
        ag += fabs(static_cast<double>(w)) * static_cast<double>(sc[u]);
    }
}

// One chunk of a long row: float64 partials of the C neighbour sums at
// partial[chunk * 8 + c] and of the Gershgorin sum at partial[chunk * 8 + C].
template <int C>
__device__ __forceinline__ void hop1_chunk(const HopArgs& a, const float* zpk) {
    __shared__ double red[kBT / kWave];
    int r, li, k0, k1, n0, ln, h0;
    chunk_range(blockIdx.x, a.long_rows, a.chunk_row, a.chunk0, a.m, r, li, k0, k1, n0, ln, h0);
    constexpr int U = kChunk / kBT;
    double acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0;
    double ag = 0;
    {
        int2 e[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int k = k0 + static_cast<int>(threadIdx.x) + u * kBT;
            int kc = k < k1 ? k : k1 - 1;
            e[u] = row_entry<false>(a.m, n0, ln, h0, kc);
            if (k >= k1) e[u].y = 0;
        }
        Vec<C> v[U];
        float sc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) load_record<C>(zpk, e[u].x, v[u], sc[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double w = static_cast<double>(bits_f(e[u].y));
#pragma unroll
            for (int c = 0; c < C; ++c) acc[c] += w * static_cast<double>(v[u].v[c]);
            ag += fabs(w) * static_cast<double>(sc[u]);
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = block_sum_f64<kBT>(acc[c], red);
    ag = block_sum_f64<kBT>(ag, red);
    if (threadIdx.x == 0) {
        double* part = a.partial + static_cast<int64_t>(blockIdx.x) * 8;
#pragma unroll
        for (int c = 0; c < C; ++c) part[c] = acc[c];
        part[C] = ag;
    }
}

// Chunk workgroups first, then short-row tiles (G lanes per row, XCD-dealt
// as in k_hop); every thread reaches the workgroup's maximum, which goes to
// wgmax[tile].
template <int C, int G, int U>
__global__ void __launch_bounds__(kBT) k_hop1_gersh(HopArgs a, const float* __restrict__ zpk,
                                                    const double* __restrict__ deg, double* __restrict__ wgmax) {
    __shared__ double red[kBT / kWave];
    if (static_cast<int>(blockIdx.x) < a.n_chunk_blocks) {
        hop1_chunk<C>(a, zpk);
        return;
    }
    const int64_t nb = static_cast<int64_t>(gridDim.x) - a.n_chunk_blocks;     // a multiple of kXcds
    const int64_t tile = xcd_tile(static_cast<int64_t>(blockIdx.x) - a.n_chunk_blocks, nb);
    const int64_t r64 = (tile * kBT + threadIdx.x) / G;
    const int l = static_cast<int>(threadIdx.x & (G - 1));
    bool valid = r64 < a.n_rows;
    const int r = valid ? static_cast<int>(r64) : 0;
    int n0 = 0, ln = 0, h0 = 0, len = 0;
    if (valid) {
        n0 = a.m.net_rp[r];
        ln = a.m.net_rp[r + 1] - n0;
        h0 = a.m.hint_rp[r];
        len = ln + (a.m.hint_rp[r + 1] - h0);
        if (len > kLongRow) valid = false;                 // group-uniform: chunk workgroups
    }
    float acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.f;
    double ag = 0;
    if (valid)
        for (int k0 = l; k0 < len; k0 += G * U) gather_batch_gersh<C, U>(a, zpk, n0, ln, h0, len, k0, G, acc, ag);
    Vec<C> sum;
#pragma unroll
    for (int c = 0; c < C; ++c) sum.v[c] = acc[c];
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
#pragma unroll
        for (int c = 0; c < C; ++c) sum.v[c] += __shfl_xor(sum.v[c], o);
        ag += __shfl_xor(ag, o);
    }
    double gv = 0;
    if (valid && l == 0) {
        vstore<C>(a.zout + static_cast<int64_t>(r) * C, sum);
        const float sr = a.scale[r];
        gv = diag_abs(sr, deg[r], a.sigma) + static_cast<double>(sr) * ag;
    }
    gv = wave_max(gv);
    __syncthreads();
    if (lane_id() == 0) red[wave_id()] = gv;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = red[0];
        for (int w = 1; w < kBT / kWave; ++w) b = red[w] > b ? red[w] : b;
        wgmax[tile] = b;
    }
}

// Long rows: one wave per row adds its chunk partials (fixed order, as
// k_hop_long), stores the unscaled neighbour sum in zout, and puts the
// row's Gershgorin value (its chunks added in order, as k_long_gersh_final)
// in lmax[li].
template <int C>
__global__ void __launch_bounds__(kBT) k_hop1_long(HopArgs a, int32_t n_long, const double* __restrict__ deg,
                                                   double* __restrict__ lmax) {
    const int64_t li = (static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x) / kWave;
    if (li >= n_long) return;
    const int r = a.long_rows[li];
    const int c0 = a.chunk0[li], c1 = a.chunk0[li + 1];
    const int l = lane_id();
    double tot[C];
#pragma unroll
    for (int c = 0; c < C; ++c) tot[c] = 0;
    for (int q = c0 + l; q < c1; q += kWave) {
#pragma unroll
        for (int c = 0; c < C; ++c) tot[c] += a.partial[static_cast<int64_t>(q) * 8 + c];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) tot[c] = wave_sum(tot[c]);
    if (l != 0) return;
    Vec<C> sum;
#pragma unroll
    for (int c = 0; c < C; ++c) sum.v[c] = static_cast<float>(tot[c]);
    vstore<C>(a.zout + static_cast<int64_t>(r) * C, sum);
    double g = 0;
    for (int q = c0; q < c1; ++q) g += a.partial[static_cast<int64_t>(q) * 8 + C];
    const float sr = a.scale[r];
    lmax[li] = diag_abs(sr, deg[r], a.sigma) + static_cast<double>(sr) * g;
}

// lambda_up = the largest of the workgroup and long-row maxima (0 if none).
__global__ void __launch_bounds__(1024) k_lam_reduce(const double* __restrict__ wgmax, int64_t nwg,
                                                     const double* __restrict__ lmax, int32_t n_long,
                                                     double* __restrict__ lam) {
    __shared__ double red[1024 / kWave];
    // eight loads in flight per lane; indexes clamped to the last value (a
    // maximum is exact in any order and repeats do not change it)
    constexpr int U = 8;
    double b = 0;
    for (int64_t i0 = threadIdx.x; i0 < nwg; i0 += U * 1024) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = wgmax[i0 + u * 1024 < nwg ? i0 + u * 1024 : nwg - 1];
#pragma unroll
        for (int u = 0; u < U; ++u) b = v[u] > b ? v[u] : b;
    }
    for (int64_t i = threadIdx.x; i < n_long; i += 1024) b = lmax[i] > b ? lmax[i] : b;
    b = wave_max(b);
    __syncthreads();
    if (lane_id() == 0) red[wave_id()] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < 1024 / kWave; ++w) m = red[w] > m ? red[w] : m;
        *lam = m;
    }
}

// The first hop's epilogue once lambda_up and the coefficients are known:
// zout holds the rows' unscaled neighbour sums, the records the rows' z.
template <int C>
__global__ void __launch_bounds__(kBT) k_hop1_epi(HopArgs a, const float* __restrict__ zpk,
                                                  const double* __restrict__ lam, double sigma,
                                                  float2* __restrict__ coef_out) {
    const int64_t r64 = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x;
    if (r64 >= a.n_rows) return;
    const int r = static_cast<int>(r64);
    RowOps<C> ops;
    ops.s = a.scale[r];
    if (coef_out) {        // the row's hop coefficients, formed here once lambda_up is known
        float cr, kr;
        hop_coef(ops.s, *lam, sigma, cr, kr);
        ops.k = make_float2(cr, kr);
        coef_out[r] = ops.k;
    } else if (a.coef) {
        ops.k = a.coef[r];
    }
    {
        const Floats<C> zr = load_floats<C>(zpk + static_cast<int64_t>(r) * pack_width<C>());
#pragma unroll
        for (int c = 0; c < C; ++c) ops.z.v[c] = zr.v[c];
    }
    if (a.band == 2) ops.acc = vload<C>(a.acc + static_cast<int64_t>(r) * C);
    ops.inst = r;          // never the last hop
    ops.flag = 0;
    const Vec<C> sum = vload<C>(a.zout + static_cast<int64_t>(r) * C);
    epilogue<C>(a, r, ops, sum);
}

// K = 0: out = (sum alpha) X on movable rows, X on fixed rows.
template <int C>
__global__ void k_identity(int32_t n_inst, const uint8_t* __restrict__ flags, const float* __restrict__ in,
                           float* __restrict__ out, float alpha_sum) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= static_cast<int64_t>(n_inst) * C) return;
    float v = in[i];
    out[i] = (flags[i / C] & AHR_NODE_FIXED) ? v : alpha_sum * v;
}

template <int C>
__global__ void k_relax(int32_t n_inst, const uint8_t* __restrict__ flags, const float* __restrict__ gc,
                        const float* __restrict__ gt, float* __restrict__ gn, float gamma) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= static_cast<int64_t>(n_inst) * C) return;
    float a = gc[i];
    gn[i] = (flags[i / C] & AHR_NODE_FIXED) ? a : (1.0f - gamma) * a + gamma * gt[i];
}

// The profiled hop time is the k_hop kernel's own (its launch carries the
// event pair; the chunk partials' k_hop_long is not part of it), so that it
// matches a kernel trace of k_hop; `bytes` are the algorithmic bytes of the whole hop.  ntiles
// column tiles of C columns each run as blockIdx.y.
template <int C, int G>
void launch_hop(const HopArgs& a, int32_t n_long_rows, double bytes, int ntiles, hipStream_t s) {
    constexpr int U = 16 / G > 8 ? 8 : (16 / G < 1 ? 1 : 16 / G);   // entries per lane per batch (16 per row, at most 8)
    int64_t tiles = grid_for(static_cast<int64_t>(a.n_rows) * G, kBT);
    tiles = (tiles + kXcds - 1) / kXcds * kXcds;                    // see xcd_tile
    int64_t blocks = a.n_chunk_blocks + tiles;
    const dim3 grid(static_cast<unsigned>(blocks), static_cast<unsigned>(ntiles));
    hipEvent_t e0, e1;
    if (prof_kernel_events(kStageHop, &e0, &e1)) {
        if (g_hop_nt)
            hipExtLaunchKernelGGL((k_hop<C, G, U, true>), grid, dim3(kBT), 0, s, e0, e1, 0, a);
        else
            hipExtLaunchKernelGGL((k_hop<C, G, U, false>), grid, dim3(kBT), 0, s, e0, e1, 0, a);
        AHR_LAUNCHED("k_hop");
        prof_kernel_done(kStageHop, e0, e1, bytes);
    } else {
        if (g_hop_nt)
            hipLaunchKernelGGL((k_hop<C, G, U, true>), grid, dim3(kBT), 0, s, a);
        else
            hipLaunchKernelGGL((k_hop<C, G, U, false>), grid, dim3(kBT), 0, s, a);
        AHR_LAUNCHED("k_hop");
    }
    if (n_long_rows > 0) {
        hipLaunchKernelGGL(k_hop_long<C>,
                           dim3(grid_for(static_cast<int64_t>(n_long_rows) * kWave, kBT), static_cast<unsigned>(ntiles)),
                           dim3(kBT), 0, s, a, n_long_rows);
        AHR_LAUNCHED("k_hop_long");
    }
}

template <int C>
void launch_hop_rb(const HopArgs& a, int32_t n_long_rows, double bytes, int ntiles, hipStream_t s) {
    int64_t tiles = (static_cast<int64_t>(a.n_rb) + kXcds - 1) / kXcds * kXcds;   // see xcd_tile
    if (tiles < kXcds) tiles = kXcds;
    const dim3 grid(static_cast<unsigned>(a.n_chunk_blocks + tiles), static_cast<unsigned>(ntiles));
    hipEvent_t e0, e1;
    if (prof_kernel_events(kStageHop, &e0, &e1)) {
        if (g_hop_nt)
            hipExtLaunchKernelGGL((k_hop_rb<C, true>), grid, dim3(kBT), 0, s, e0, e1, 0, a);
        else
            hipExtLaunchKernelGGL((k_hop_rb<C, false>), grid, dim3(kBT), 0, s, e0, e1, 0, a);
        AHR_LAUNCHED("k_hop_rb");
        prof_kernel_done(kStageHop, e0, e1, bytes);
    } else {
        if (g_hop_nt)
            hipLaunchKernelGGL((k_hop_rb<C, true>), grid, dim3(kBT), 0, s, a);
        else
            hipLaunchKernelGGL((k_hop_rb<C, false>), grid, dim3(kBT), 0, s, a);
        AHR_LAUNCHED("k_hop_rb");
    }
    if (n_long_rows > 0) {
        hipLaunchKernelGGL(k_hop_long<C>,
                           dim3(grid_for(static_cast<int64_t>(n_long_rows) * kWave, kBT), static_cast<unsigned>(ntiles)),
                           dim3(kBT), 0, s, a, n_long_rows);
        AHR_LAUNCHED("k_hop_long");
    }
}

template <int C>
void hop_dispatch(const HopArgs& a, int lanes, int32_t n_long_rows, double bytes, int ntiles, hipStream_t s) {
    switch (lanes) {
        case AHR_HOP_ROW_BLOCK: launch_hop_rb<C>(a, n_long_rows, bytes, ntiles, s); break;
        case 1: launch_hop<C, 1>(a, n_long_rows, bytes, ntiles, s); break;
        case 2: launch_hop<C, 2>(a, n_long_rows, bytes, ntiles, s); break;
        case 4: launch_hop<C, 4>(a, n_long_rows, bytes, ntiles, s); break;
        case 8: launch_hop<C, 8>(a, n_long_rows, bytes, ntiles, s); break;
        case 16: launch_hop<C, 16>(a, n_long_rows, bytes, ntiles, s); break;
        case 32: launch_hop<C, 32>(a, n_long_rows, bytes, ntiles, s); break;
        default: launch_hop<C, 64>(a, n_long_rows, bytes, ntiles, s); break;
    }
}

template <int C>
void expand_signal(Graph& g, const float* in, bool band0, float alpha0, hipStream_t s, float* zpk = nullptr) {
    ExpandArgs e = expand_args(g);
    e.in = in;
    e.z0 = g.z0.p;
    e.zpk = zpk;
    e.acc = g.acc.p;
    e.alpha0 = alpha0;
    e.band0 = band0 ? 1 : 0;
    e.ct = C;
    e.tile_stride = static_cast<int64_t>(g.n_tot) * C;
    ProfScope ps(kStageExpand, s);
    const int32_t nbig = g.n_star ? g.n_big_stars : 0;
    const int32_t bstar =
        g.n_star ? static_cast<int32_t>(grid_for(static_cast<int64_t>(g.n_star) * kStarLanes, kBT)) : 0;
    const int64_t blocks = static_cast<int64_t>(nbig) + bstar + grid_for(g.n_tot, kBT);
    hipLaunchKernelGGL((k_expand_all<C, kStarLanes>), dim3(static_cast<unsigned>(blocks)), dim3(kBT), 0, s, e,
                       g.n_star, g.big_stars.p, nbig, bstar);
    AHR_LAUNCHED("k_expand_all");
}

ChainView chain_view(Graph& g, const ahr_filter_spec& spec, hipStream_t s) {
    ChainView v;
    v.net_rp = g.xnet_rp.p;
    v.net_ent = net_entries(g, s);
    v.hint_rp = g.xhint_rp.p;
    v.hint_ent = g.xhint_ent.p;
    v.scale = g.scale.p;
    v.coef = g.coef.p;
    v.lam = g.lam.p;
    v.sigma = spec.sigma;
    v.flags = g.nl.node_flags;
    v.perm = g.perm.p;
    v.long_rows = g.rc.long_rows.p;
    v.chunk_row = g.rc.chunk_row.p;
    v.chunk0 = g.rc.long_chunk0.p;
    v.partial = g.rc.partial.p;
    v.rb = g.rc.rb.p;
    v.n_tot = g.n_tot;
    v.n_inst = g.n_inst;
    v.n_long = g.rc.n_long;
    v.n_long_inst = g.rc.n_long_inst;
    v.n_chunks = g.rc.n_chunks;
    v.n_chunks_inst = g.rc.n_chunks_inst;
    v.n_rb = g.rc.n_rb;
    v.n_rb_inst = g.rc.n_rb_inst;
    v.nnz_inst = g.rc.nnz_inst;
    v.nnz_all = g.rc.nnz_net_all + g.rc.nnz_hint_all;
    v.z0 = g.z0.p;
    v.z1 = g.z1.p;
    v.acc = g.acc.p;
    return v;
}

HopArgs hop_args(const ChainView& v, const float* in, float* out, int ncols) {
    HopArgs h;
    h.m = RowRef{v.net_rp, v.net_ent, v.hint_rp, v.hint_ent};
    h.perm = v.perm;
    h.scale = v.scale;
    h.coef = v.coef;
    h.lam = v.lam;
    h.sigma = v.sigma;
    h.acc = v.acc;
    h.gin = in;
    h.out = out;
    h.flags = v.flags;
    h.long_rows = v.long_rows;
    h.chunk_row = v.chunk_row;
    h.chunk0 = v.chunk0;
    h.partial = v.partial;
    h.rb = v.rb;
    h.n_rb = 0;
    h.alpha_sum = 0.f;
    h.band = 0;
    h.alpha = 0.f;
    h.last = 0;
    h.zin = nullptr;
    h.zout = nullptr;
    h.n_rows = 0;
    h.n_chunk_blocks = 0;
    h.tile_stride = 0;
    h.ldo = ncols;
    h.col0 = 0;
    return h;
}

// Algorithmic bytes of one hop launch over C columns: row pointers,
// (column, weight) entries, one read of the gathered signal, the row
// writes, the band accumulator.
double hop_bytes(const ChainView& v, const HopArgs& h, int C) {
    const double R = h.n_rows;
    const double E = h.n_rows < v.n_tot ? static_cast<double>(v.nnz_inst) : static_cast<double>(v.nnz_all);
    double acc_b = 0;
    if (h.band == 1) acc_b = h.last ? 0 : 4.0 * C * R;
    if (h.band == 2) acc_b = h.last ? 4.0 * C * R : 8.0 * C * R;
    return 4.0 * (R + 1) + 8.0 * E + 4.0 * C * static_cast<double>(v.n_tot) + 4.0 * C * R + acc_b;
}

// The unpinned chain y_j = T^j X for j = 1..3 (scaled coordinates, into
// g.zh[j-1]); the third hop only for the instance rows.
template <int C>
void hops_c(Graph& g, const ahr_filter_spec& spec, const float* in, int lanes, hipStream_t s) {
    const int64_t N = g.n_tot;
    g.z0.ensure(static_cast<size_t>(N) * C, s);
    g.acc.ensure(static_cast<size_t>(N) * C, s);
    for (auto& z : g.zh) z.ensure(static_cast<size_t>(N) * C, s);
    expand_signal<C>(g, in, false, 0.f, s);
    const ChainView v = chain_view(g, spec, s);
    HopArgs h = hop_args(v, in, nullptr, C);
    const float* zin = g.z0.p;
    for (int j = 0; j < 3; ++j) {
        h.zin = zin;
        h.zout = g.zh[j].p;
        const bool inst_only = j == 2;
        h.n_rows = inst_only ? v.n_inst : v.n_tot;
        h.n_chunk_blocks = inst_only ? v.n_chunks_inst : v.n_chunks;
        h.n_rb = inst_only ? v.n_rb_inst : v.n_rb;
        hop_dispatch<C>(h, lanes, inst_only ? v.n_long_inst : v.n_long, hop_bytes(v, h, C), 1, s);
        zin = g.zh[j].p;
    }
}

// Weight of power j in the bank (sum over bands with k_b = j).
float alpha_at(const ahr_filter_spec& spec, int j, bool& is_band) {
    float a = 0.f;
    is_band = false;
    for (int b = 0; b < spec.nbands; ++b)
        if (spec.k[b] == j) {
            a += spec.alpha[b];
            is_band = true;
        }
    return a;
}

// What the first hop needs to form lambda_up itself (k_hop1_gersh).
struct Hop1Gersh {
    const float* zpk;   // the expanded signal as first-hop records
    const double* deg;
    double* gmax;       // one slot per short-row workgroup, then one per long row
    double* lam;
    float2* coef;
};

// The first hop with the Gershgorin bound (4 lanes per short row).
template <int C>
void hop1_gersh(const ChainView& v, HopArgs h, const Hop1Gersh& f, hipStream_t s) {
    constexpr int G = 4, U = 4;
    int64_t tiles = grid_for(static_cast<int64_t>(h.n_rows) * G, kBT);
    tiles = (tiles + kXcds - 1) / kXcds * kXcds;                    // see xcd_tile
    hipLaunchKernelGGL((k_hop1_gersh<C, G, U>), dim3(static_cast<unsigned>(h.n_chunk_blocks + tiles)), dim3(kBT), 0,
                       s, h, f.zpk, f.deg, f.gmax);
    AHR_LAUNCHED("k_hop1_gersh");
    if (v.n_long > 0) {
        hipLaunchKernelGGL(k_hop1_long<C>, dim3(grid_for(static_cast<int64_t>(v.n_long) * kWave, kBT)), dim3(kBT), 0, s,
                           h, v.n_long, f.deg, f.gmax + tiles);
        AHR_LAUNCHED("k_hop1_long");
    }
    hipLaunchKernelGGL(k_lam_reduce, dim3(1), dim3(1024), 0, s, f.gmax, tiles, f.gmax + tiles, v.n_long, f.lam);
    AHR_LAUNCHED("k_lam_reduce");
    // the epilogue forms every row's coefficients when it covers every row
    const bool fused = h.n_rows == v.n_tot;
    if (!fused) hop_coefs(v.n_tot, v.scale, f.lam, v.sigma, f.coef, s);
    hipLaunchKernelGGL(k_hop1_epi<C>, dim3(grid_for(h.n_rows, kBT)), dim3(kBT), 0, s, h, f.zpk, f.lam, v.sigma,
                       fused ? f.coef : nullptr);
    AHR_LAUNCHED("k_hop1_epi");
}

// Hops 1..k_max over column tiles of CT columns (C / CT tiles); with f, the
// first hop also forms lambda_up (needs CT = C <= 4, k_max >= 2).
template <int C, int CT>
void chain_c(const ChainView& v, const ahr_filter_spec& spec, const float* in, float* out, int lanes, hipStream_t s,
             const Hop1Gersh* f = nullptr) {
    float alpha_sum = 0.f;
    const int kmax = spec_kmax(spec, &alpha_sum);
    bool b0;
    alpha_at(spec, 0, b0);
    HopArgs h = hop_args(v, in, out, C);
    h.alpha_sum = alpha_sum;
    h.tile_stride = static_cast<int64_t>(v.n_tot) * CT;
    bool has_acc = b0;
    float* zin = v.z0;
    float* zout = v.z1;
    for (int j = 1; j <= kmax; ++j) {
        bool isb;
        float aj = alpha_at(spec, j, isb);
        h.zin = zin;
        h.zout = zout;
        h.last = j == kmax;
        h.band = isb ? (has_acc ? 2 : 1) : 0;
        h.alpha = aj;
        h.n_rows = h.last ? v.n_inst : v.n_tot;
        h.n_chunk_blocks = h.last ? v.n_chunks_inst : v.n_chunks;
        h.n_rb = h.last ? v.n_rb_inst : v.n_rb;
        if (f && j == 1) {
            if constexpr (CT == C && C <= 4) {
                ProfScope ps(kStageNorm, s);
                hop1_gersh<C>(v, h, *f, s);
            } else {
                throw Error{AHR_EINVAL, "first-hop bound needs one column tile of at most 4 columns"};
            }
        } else {
            hop_dispatch<CT>(h, lanes, h.last ? v.n_long_inst : v.n_long, hop_bytes(v, h, C), C / CT, s);
        }
        has_acc = has_acc || isb;
        float* t = zin;
        zin = zout;
        zout = t;
    }
}

template <int C>
void chain_tiles(const ChainView& v, const ahr_filter_spec& spec, const float* in, float* out, int lanes, int ct,
                 hipStream_t s) {
    if (ct == C) return chain_c<C, C>(v, spec, in, out, lanes, s);
    if constexpr (C >= 2) {
        if (ct == 1) return chain_c<C, 1>(v, spec, in, out, lanes, s);
    }
    if constexpr (C >= 4) {
        if (ct == 2) return chain_c<C, 2>(v, spec, in, out, lanes, s);
    }
    if constexpr (C >= 8) {
        if (ct == 4) return chain_c<C, 4>(v, spec, in, out, lanes, s);
    }
    throw Error{AHR_EINVAL, "column tile must divide the column count"};
}

template <int C>
void filter_c(Graph& g, const ahr_filter_spec& spec, const float* in, float* out, int lanes, hipStream_t s,
              bool hop1_bound = false) {
    const int64_t N = g.n_tot;
    float alpha_sum = 0.f;
    const int kmax = spec_kmax(spec, &alpha_sum);
    if (kmax == 0) {
        int64_t n = static_cast<int64_t>(g.n_inst) * C;
        hipLaunchKernelGGL((k_identity<C>), dim3(grid_for(n, kBT)), dim3(kBT), 0, s, g.n_inst, g.nl.node_flags, in, out,
                           alpha_sum);
        AHR_LAUNCHED("k_identity");
        return;
    }
    g.z0.ensure(static_cast<size_t>(N) * C, s);
    g.z1.ensure(static_cast<size_t>(N) * C, s);
    g.acc.ensure(static_cast<size_t>(N) * C, s);
    bool b0;
    float a0 = alpha_at(spec, 0, b0);
    if (hop1_bound) {
        if constexpr (C <= 4) {
            g.zpk.ensure(static_cast<size_t>(N) * pack_width<C>(), s);
            expand_signal<C>(g, in, b0, a0, s, g.zpk.p);
        }
        const Hop1Gersh f{g.zpk.p, g.deg.p, g.gmax.p, g.lam.p, g.coef.p};
        chain_c<C, C>(chain_view(g, spec, s), spec, in, out, lanes, s, &f);
    } else {
        expand_signal<C>(g, in, b0, a0, s);
        chain_c<C, C>(chain_view(g, spec, s), spec, in, out, lanes, s);
    }
}

template <int C>
void expand_batch_c(const ExpandArgs* d, const int32_t* blk0, int32_t n_blocks, const int32_t* sblk0,
                    int32_t n_star_blocks, const int32_t* big, int32_t n_big, int32_t ng, const float* in,
                    hipStream_t s) {
    hipLaunchKernelGGL((k_expand_batch<C>), dim3(static_cast<unsigned>(n_blocks)), dim3(kBT), 0, s, d, blk0, ng, in);
    AHR_LAUNCHED("k_expand_batch");
    if (n_star_blocks > 0) {     // here: the total star count of the batch
        hipLaunchKernelGGL((k_expand_star_batch<C, kStarLanes>),
                           dim3(grid_for(static_cast<int64_t>(n_star_blocks) * kStarLanes, kBT)), dim3(kBT), 0, s, d,
                           sblk0, ng, n_star_blocks, in);
        AHR_LAUNCHED("k_expand_star_batch");
        if (n_big) {
            hipLaunchKernelGGL((k_expand_big_star_batch<C>), dim3(static_cast<unsigned>(n_big)), dim3(kBT), 0, s, d,
                               sblk0, ng, big, in);
            AHR_LAUNCHED("k_expand_big_star_batch");
        }
    }
}

}  // namespace

// Row classes in two halves around the read of their counts: the first
// launches the flags, scans and the read; whatever the caller queues before
// the second runs while the host waits for the counts.  `extra`, when given,
// is one more device word read with them (to *extra_out).
struct RowClassScratch {
    DevBuf<int32_t> is_long, rank, nch, cscan;
};

static void row_classes_begin(const int32_t* net_rp, const int32_t* hint_rp, int32_t N, int32_t n_inst,
                              RowClassScratch& t, DevBuf<int64_t>& scan_tmp, hipStream_t s,
                              const int32_t* extra = nullptr) {
    const size_t n1 = static_cast<size_t>(N) + 1;
    t.is_long.ensure(n1, s);
    t.nch.ensure(n1, s);
    hipLaunchKernelGGL(k_row_chunks, dim3(grid_for(N, kBT)), dim3(kBT), 0, s, N, net_rp, hint_rp, t.is_long.p,
                       t.nch.p);
    AHR_LAUNCHED("k_row_chunks");
    t.rank.ensure(n1, s);
    t.cscan.ensure(n1, s);
    scan_tmp.ensure(scan_tmp_elems(N), s);
    scan_i32_to_i32(t.is_long.p, t.rank.p, N, scan_tmp.p, s);
    scan_i32_to_i32(t.nch.p, t.cscan.p, N, scan_tmp.p, s);
    std::vector<const int32_t*> words{t.rank.p + N,  t.rank.p + n_inst, t.cscan.p + N, t.cscan.p + n_inst,
                                      net_rp + n_inst, hint_rp + n_inst, net_rp + N, hint_rp + N};
    if (extra) words.push_back(extra);
    read_scalars_begin(words, s);
}

static void row_classes_end(int32_t N, RowClasses& rc, RowClassScratch& t, hipStream_t s,
                            int32_t* extra_out = nullptr) {
    int32_t v[9];
    read_scalars_end(v, extra_out ? 9 : 8);
    if (extra_out) *extra_out = v[8];
    rc.nnz_net_all = v[6];
    rc.nnz_hint_all = v[7];
    rc.n_long = v[0];
    rc.n_long_inst = v[1];
    rc.n_chunks = v[2];
    rc.n_chunks_inst = v[3];
    rc.nnz_inst = static_cast<int64_t>(v[4]) + v[5];
    rc.has_rb = 0;
    rc.long_rows.ensure(static_cast<size_t>(rc.n_long) + 1, s);
    list_rows(t.is_long.p, t.rank.p, N, rc.long_rows.p, s);
    rc.long_chunk0.ensure(static_cast<size_t>(rc.n_long) + 1, s);
    hipLaunchKernelGGL(k_long_chunk0, dim3(grid_for(static_cast<int64_t>(rc.n_long) + 1, kBT)), dim3(kBT), 0, s,
                       rc.n_long, rc.long_rows.p, t.cscan.p, rc.n_chunks, rc.long_chunk0.p);
    AHR_LAUNCHED("k_long_chunk0");
    rc.chunk_row.ensure(static_cast<size_t>(rc.n_chunks) + 1, s);
    if (rc.n_long) {
        hipLaunchKernelGGL(k_chunk_rows, dim3(rc.n_long), dim3(kBT), 0, s, rc.n_long, rc.long_chunk0.p,
                           rc.chunk_row.p);
        AHR_LAUNCHED("k_chunk_rows");
    }
    rc.partial.ensure(static_cast<size_t>(rc.n_chunks) * 8 + 8, s);
    t.is_long.release(s);
    t.rank.release(s);
    t.nch.release(s);
    t.cscan.release(s);
}

void row_classes(const int32_t* net_rp, const int32_t* hint_rp, int32_t N, int32_t n_inst, RowClasses& rc,
                 DevBuf<int64_t>& scan_tmp, hipStream_t s) {
    RowClassScratch t;
    row_classes_begin(net_rp, hint_rp, N, n_inst, t, scan_tmp, s);
    row_classes_end(N, rc, t, s);
}

void row_blocks(const int32_t* net_rp, const int32_t* hint_rp, int32_t N, int32_t n_inst, RowClasses& rc,
                DevBuf<int64_t>& scan_tmp, hipStream_t s) {
    if (rc.has_rb) return;
    DevBuf<int32_t> is_long, st, en, srank, erank, starts, ends;
    const size_t n1 = static_cast<size_t>(N) + 1;
    is_long.ensure(n1, s);
    hipLaunchKernelGGL(k_row_len, dim3(grid_for(N, kBT)), dim3(kBT), 0, s, N, net_rp, hint_rp, is_long.p);
    AHR_LAUNCHED("k_row_len");
    st.ensure(n1, s);
    en.ensure(n1, s);
    hipLaunchKernelGGL(k_rb_marks, dim3(grid_for(N, kBT)), dim3(kBT), 0, s, N, n_inst, net_rp, hint_rp, is_long.p, st.p,
                       en.p);
    AHR_LAUNCHED("k_rb_marks");
    srank.ensure(n1, s);
    erank.ensure(n1, s);
    scan_tmp.ensure(scan_tmp_elems(N), s);
    scan_i32_to_i32(st.p, srank.p, N, scan_tmp.p, s);
    scan_i32_to_i32(en.p, erank.p, N, scan_tmp.p, s);
    int32_t t[2];
    read_scalars({srank.p + N, srank.p + n_inst}, t, s);
    rc.n_rb = t[0];
    rc.n_rb_inst = t[1];
    starts.ensure(static_cast<size_t>(rc.n_rb) + 1, s);
    ends.ensure(static_cast<size_t>(rc.n_rb) + 1, s);
    list_rows(st.p, srank.p, N, starts.p, s);
    list_rows(en.p, erank.p, N, ends.p, s);
    rc.rb.ensure(2 * static_cast<size_t>(rc.n_rb) + 2, s);
    if (rc.n_rb) {
        hipLaunchKernelGGL(k_rb_desc, dim3(grid_for(rc.n_rb, kBT)), dim3(kBT), 0, s, rc.n_rb, starts.p, ends.p, net_rp,
                           hint_rp, rc.rb.p);
        AHR_LAUNCHED("k_rb_desc");
    }
    rc.has_rb = 1;
    for (auto* b : {&is_long, &st, &en, &srank, &erank, &starts, &ends}) b->release(s);
}

void hop_coefs(int32_t n, const float* scale, const double* lam, double sigma, float2* coef, hipStream_t s) {
    hipLaunchKernelGGL(k_coef, dim3(grid_for(n, kBT)), dim3(kBT), 0, s, n, scale, lam, sigma, coef);
    AHR_LAUNCHED("k_coef");
}

ExpandArgs expand_args(const Graph& g) {
    ExpandArgs e;
    e.in = nullptr;
    e.in_off = 0;
    e.perm = g.perm.p;
    e.iperm = g.iperm.p;
    e.xmpin = g.xmpin.p;
    e.xstar_net = g.xstar_net.p;
    e.scale = g.scale.p;
    e.z0 = nullptr;
    e.zpk = nullptr;
    e.acc = nullptr;
    e.alpha0 = 0.f;
    e.band0 = 0;
    e.n_inst = g.n_inst;
    e.first_mpin = g.first_mpin;
    e.first_star = g.first_star;
    e.first_mvirt = g.first_mvirt;
    e.first_bvirt = g.first_bvirt;
    e.n_tot = g.n_tot;
    e.row_inst0 = 0;
    e.row_aux0 = g.n_inst;
    e.ct = 1;
    e.tile_stride = 0;
    e.mpin_owner = g.mpin_owner.p;
    e.mpin_pin = g.mpin_pin.p;
    e.pin_off = g.nl.pin_off;
    e.star_net = g.star_net.p;
    e.net_ptr = g.nl.net_ptr;
    e.pin_node = g.nl.pin_node;
    e.pin_node_x = g.pin_node_x.p;
    e.macro_ids = g.macro_ids.p;
    e.nbx = g.hp.nbx;
    e.xl = g.nl.die[0];
    e.yl = g.nl.die[1];
    e.bw = (static_cast<double>(g.nl.die[2]) - static_cast<double>(g.nl.die[0])) / g.hp.nbx;
    e.bh = (static_cast<double>(g.nl.die[3]) - static_cast<double>(g.nl.die[1])) / g.hp.nby;
    return e;
}

void expand_batch(const ExpandArgs* d, const int32_t* blk0, int32_t n_blocks, const int32_t* sblk0,
                  int32_t n_star_blocks, const int32_t* big, int32_t n_big, int32_t ng, const float* in,
                  int32_t ncols, hipStream_t s) {
    switch (ncols) {
        case 1: expand_batch_c<1>(d, blk0, n_blocks, sblk0, n_star_blocks, big, n_big, ng, in, s); break;
        case 2: expand_batch_c<2>(d, blk0, n_blocks, sblk0, n_star_blocks, big, n_big, ng, in, s); break;
        case 4: expand_batch_c<4>(d, blk0, n_blocks, sblk0, n_star_blocks, big, n_big, ng, in, s); break;
        case 8: expand_batch_c<8>(d, blk0, n_blocks, sblk0, n_star_blocks, big, n_big, ng, in, s); break;
        default: throw Error{AHR_EUNSUPPORTED, "ncols must be 1, 2, 4 or 8"};
    }
}

void run_chain(const ChainView& v, const ahr_filter_spec& spec, const float* in, float* out, int32_t ncols, int lanes,
               int ct, hipStream_t s) {
    switch (ncols) {
        case 1: chain_tiles<1>(v, spec, in, out, lanes, ct, s); break;
        case 2: chain_tiles<2>(v, spec, in, out, lanes, ct, s); break;
        case 4: chain_tiles<4>(v, spec, in, out, lanes, ct, s); break;
        case 8: chain_tiles<8>(v, spec, in, out, lanes, ct, s); break;
        default: throw Error{AHR_EUNSUPPORTED, "ncols must be 1, 2, 4 or 8"};
    }
}

int32_t spec_kmax(const ahr_filter_spec& spec, float* alpha_sum) {
    int32_t kmax = 0;
    float as = 0.f;
    for (int b = 0; b < spec.nbands; ++b) {
        kmax = spec.k[b] > kmax ? spec.k[b] : kmax;
        as += spec.alpha[b];
    }
    if (alpha_sum) *alpha_sum = as;
    return kmax;
}

namespace {

bool norm_current(const Graph& g, const ahr_filter_spec& spec) {
    return g.norm_version == g.hint_version && g.norm_sigma == spec.sigma && g.norm_mode == spec.lambda_mode &&
           g.norm_fixed == spec.lambda_fixed;
}

void norm_done(Graph& g, const ahr_filter_spec& spec) {
    g.norm_version = g.hint_version;
    g.norm_sigma = spec.sigma;
    g.norm_mode = spec.lambda_mode;
    g.norm_fixed = spec.lambda_fixed;
}

// Row classes, degrees, scales and hint sums of the operator.
void normalise_degrees(Graph& g, const ahr_filter_spec& spec, hipStream_t s) {
    const int32_t N = g.n_tot;
    // a netlist row's absolute degree is its qdeg: these kernels read the
    // netlist rows' lengths and the hint entries only
    RowRef m{g.xnet_rp.p, nullptr, g.xhint_rp.p, g.xhint_ent.p};

    // the row classes' counts are read while the short rows' degrees run
    RowClassScratch rct;
    const bool new_rows = g.rows_version != g.hint_version;
    // the layout's locality verdict rides along with the first counts
    const bool want_loc = new_rows && g.hop_local < 0 && g.loc_flag.p;
    if (new_rows)
        row_classes_begin(g.xnet_rp.p, g.xhint_rp.p, N, g.n_inst, rct, g.scan_tmp, s,
                          want_loc ? g.loc_flag.p : nullptr);

    const double sigma = spec.sigma;
    g.deg.ensure(static_cast<size_t>(N) + 1, s);
    g.scale.ensure(static_cast<size_t>(N) + 1, s);
    g.hsum.ensure(static_cast<size_t>(N) + 1, s);
    g.lam.ensure(1, s);
    g.coef.ensure(static_cast<size_t>(N) + 1, s);
    constexpr int G = 4;
    // cell rows from the hint build's sums when it formed them for this
    // hint version, then the other rows from their entries
    const int32_t r0 = g.habs_version == g.hint_version ? g.n_inst : 0;
    const int32_t cell_blocks = r0 ? static_cast<int32_t>(grid_for(r0, kBT)) : 0;
    const int64_t short_blocks = N > r0 ? grid_for(static_cast<int64_t>(N - r0) * G, kBT) : 0;
    if (cell_blocks + short_blocks) {
        hipLaunchKernelGGL(k_deg_rows<G>, dim3(static_cast<unsigned>(cell_blocks + short_blocks)), dim3(kBT), 0, s,
                           r0, N, cell_blocks, m, g.xqdeg.p, g.xhabs.p, g.xhsg.p, sigma, g.deg.p, g.scale.p,
                           g.hsum.p);
        AHR_LAUNCHED("k_deg_rows");
    }
    if (new_rows) {
        int32_t loc = 1;
        row_classes_end(N, g.rc, rct, s, want_loc ? &loc : nullptr);
        if (want_loc) g.hop_local = loc ? 1 : 0;
        g.rows_version = g.hint_version;
        g.nnz_net = static_cast<int32_t>(g.rc.nnz_net_all);
        g.nnz_hint = static_cast<int32_t>(g.rc.nnz_hint_all);
    }
    if (g.rc.n_long) {
        hipLaunchKernelGGL(k_chunk_absdeg, dim3(g.rc.n_chunks), dim3(kBT), 0, s, m, g.rc.long_rows.p, g.rc.chunk_row.p,
                           g.rc.long_chunk0.p, g.rc.partial.p);
        AHR_LAUNCHED("k_chunk_absdeg");
        hipLaunchKernelGGL(k_long_deg_final, dim3(grid_for(g.rc.n_long, kBT)), dim3(kBT), 0, s, g.rc.n_long, g.rc.long_rows.p,
                           g.rc.long_chunk0.p, g.rc.partial.p, g.xqdeg.p, sigma, g.deg.p, g.scale.p, g.hsum.p);
        AHR_LAUNCHED("k_long_deg_final");
    }
}

}  // namespace

void normalise(Graph& g, const ahr_filter_spec& spec, hipStream_t s) {
    if (norm_current(g, spec)) return;
    ProfScope ps(kStageNorm, s);
    const int32_t N = g.n_tot;
    normalise_degrees(g, spec, s);
    const double sigma = spec.sigma;
    constexpr int G = 4;
    if (spec.lambda_mode == AHR_LAMBDA_FIXED) {
        hipLaunchKernelGGL(k_set_f64, dim3(1), dim3(1), 0, s, g.lam.p, static_cast<double>(spec.lambda_fixed));
        AHR_LAUNCHED("k_set_f64");
    } else {
        hipLaunchKernelGGL(k_set_f64, dim3(1), dim3(1), 0, s, g.lam.p, 0.0);
        AHR_LAUNCHED("k_set_f64");
        const RowRef m{g.xnet_rp.p, net_entries(g, s), g.xhint_rp.p, g.xhint_ent.p};
        hipLaunchKernelGGL(k_gersh_short<G>, dim3(kGershGrid), dim3(kBT), 0, s, N, m,
                           g.deg.p, g.scale.p, sigma, g.lam.p);
        AHR_LAUNCHED("k_gersh_short");
        if (g.rc.n_long) {
            hipLaunchKernelGGL(k_chunk_gersh, dim3(g.rc.n_chunks), dim3(kBT), 0, s, m, g.rc.long_rows.p, g.rc.chunk_row.p,
                               g.rc.long_chunk0.p, g.scale.p, g.rc.partial.p);
            AHR_LAUNCHED("k_chunk_gersh");
            hipLaunchKernelGGL(k_long_gersh_final, dim3(grid_for(g.rc.n_long, kBT)), dim3(kBT), 0, s, g.rc.n_long,
                               g.rc.long_rows.p, g.rc.long_chunk0.p, g.rc.partial.p, g.deg.p, g.scale.p, sigma, g.lam.p);
            AHR_LAUNCHED("k_long_gersh_final");
        }
    }
    hop_coefs(N, g.scale.p, g.lam.p, sigma, g.coef.p, s);
    norm_done(g, spec);
}

int g_hop_lanes = AHR_HOP_AUTO;   // lanes per short row (set by the tuner)
int g_hop_nt = 0;                 // non-temporal entry loads

// The hop's launch shape on graph g: the tuned one, or under AHR_HOP_AUTO 4
// lanes in a local order and the row-block form in one whose gathers mostly
// miss (read with the first row classes, so known once g is normalised).
static int hop_lanes(const Graph& g) {
    if (g_hop_lanes != AHR_HOP_AUTO) return g_hop_lanes;
    return g.hop_local == 0 ? AHR_HOP_ROW_BLOCK : 4;
}

void run_filter(Graph& g, const ahr_filter_spec& spec, const float* in, float* out, int32_t ncols, hipStream_t s) {
    // a first filter on new hints with the Gershgorin bound forms the bound
    // in its first hop (4-lane form, at most 4 columns, order >= 2)
    const bool hop1_bound = !norm_current(g, spec) && spec.lambda_mode != AHR_LAMBDA_FIXED &&
                            (g_hop_lanes == 4 || g_hop_lanes == AHR_HOP_AUTO) && ncols <= 4 &&
                            spec_kmax(spec, nullptr) >= 2;
    if (hop1_bound) {
        {
            ProfScope ps(kStageNorm, s);
            normalise_degrees(g, spec, s);
        }
        const int64_t tiles = (grid_for(static_cast<int64_t>(g.n_tot) * 4, kBT) + kXcds - 1) / kXcds * kXcds;
        g.gmax.ensure(static_cast<size_t>(tiles + g.rc.n_long) + 1, s);
    } else {
        normalise(g, spec, s);
    }
    const int lanes = hop_lanes(g);
    if (lanes == AHR_HOP_ROW_BLOCK) row_blocks(g.xnet_rp.p, g.xhint_rp.p, g.n_tot, g.n_inst, g.rc, g.scan_tmp, s);
    switch (ncols) {
        case 1: filter_c<1>(g, spec, in, out, lanes, s, hop1_bound); break;
        case 2: filter_c<2>(g, spec, in, out, lanes, s, hop1_bound); break;
        case 4: filter_c<4>(g, spec, in, out, lanes, s, hop1_bound); break;
        case 8: filter_c<8>(g, spec, in, out, lanes, s, false); break;
        default: throw Error{AHR_EUNSUPPORTED, "ncols must be 1, 2, 4 or 8"};
    }
    if (hop1_bound) norm_done(g, spec);
}

void run_hops(Graph& g, const ahr_filter_spec& spec, const float* in, int32_t ncols, hipStream_t s) {
    normalise(g, spec, s);
    const int lanes = hop_lanes(g);
    if (lanes == AHR_HOP_ROW_BLOCK) row_blocks(g.xnet_rp.p, g.xhint_rp.p, g.n_tot, g.n_inst, g.rc, g.scan_tmp, s);
    switch (ncols) {
        case 1: hops_c<1>(g, spec, in, lanes, s); break;
        case 2: hops_c<2>(g, spec, in, lanes, s); break;
        case 4: hops_c<4>(g, spec, in, lanes, s); break;
        case 8: hops_c<8>(g, spec, in, lanes, s); break;
        default: throw Error{AHR_EUNSUPPORTED, "ncols must be 1, 2, 4 or 8"};
    }
}

void relax(Graph& g, const float* gcur, const float* gt, float* gnext, int32_t ncols, float gamma, hipStream_t s) {
    ProfScope ps(kStageRelax, s);
    int64_t n = static_cast<int64_t>(g.n_inst) * ncols;
    switch (ncols) {
        case 1: hipLaunchKernelGGL(k_relax<1>, dim3(grid_for(n, kBT)), dim3(kBT), 0, s, g.n_inst, g.nl.node_flags, gcur, gt, gnext, gamma); break;
        case 2: hipLaunchKernelGGL(k_relax<2>, dim3(grid_for(n, kBT)), dim3(kBT), 0, s, g.n_inst, g.nl.node_flags, gcur, gt, gnext, gamma); break;
        case 4: hipLaunchKernelGGL(k_relax<4>, dim3(grid_for(n, kBT)), dim3(kBT), 0, s, g.n_inst, g.nl.node_flags, gcur, gt, gnext, gamma); break;
        case 8: hipLaunchKernelGGL(k_relax<8>, dim3(grid_for(n, kBT)), dim3(kBT), 0, s, g.n_inst, g.nl.node_flags, gcur, gt, gnext, gamma); break;
        default: throw Error{AHR_EUNSUPPORTED, "ncols must be 1, 2, 4 or 8"};
    }
    AHR_LAUNCHED("k_relax");
}

}  // namespace ahr
