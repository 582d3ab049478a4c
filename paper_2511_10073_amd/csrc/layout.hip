// Execution layout of the filter.  Instance ids arrive in netlist order,
// which carries no locality, so neighbour gathers of the SpMM hop would each
// touch a different cache line.  The filter therefore streams rows in an
// execution order: instances sorted by a stable bucket sort on the Z-order
// (Morton) key of their position on a 128 x 128 grid over the die, columns
// renumbered to match; added nodes (macro pins, stars, virtual nodes) keep
// their canonical ids.  The netlist rows are copied into that order (entry
// order within a row kept, so the summation order is fixed by the inputs);
// the hint rows are built in it directly.  The canonical netlist CSR stays
// for export; the order is set once per graph from the first placement seen.
#include "ahr_internal.hpp"
#include "device_util.hpp"

namespace ahr {

namespace {

constexpr int kBT = 256;
constexpr int kGridBits = 7;     // 128 x 128 layout grid -> 14-bit keys

__device__ __forceinline__ int interleave7(int x, int y) {
    int k = 0;
#pragma unroll
    for (int b = 0; b < kGridBits; ++b) k |= (((x >> b) & 1) << (2 * b)) | (((y >> b) & 1) << (2 * b + 1));
    return k;
}

__global__ void k_layout_keys(const float* __restrict__ pos, int ncols, int32_t n, float xl, float yl, float sx,
                              float sy, int32_t* __restrict__ key) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int m = (1 << kGridBits) - 1;
    float fx = floorf((pos[i * ncols] - xl) * sx);
    float fy = floorf((pos[i * ncols + 1] - yl) * sy);
    int gx = !(fx > 0.f) ? 0 : (fx >= static_cast<float>(m) ? m : static_cast<int>(fx));
    int gy = !(fy > 0.f) ? 0 : (fy >= static_cast<float>(m) ? m : static_cast<int>(fy));
    key[i] = interleave7(gx, gy);
}

__global__ void k_iperm(const int32_t* __restrict__ perm, int32_t n, int32_t* __restrict__ iperm) {
    int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r < n) iperm[perm[r]] = static_cast<int32_t>(r);
}

__device__ __forceinline__ int src_row(int r, int n_inst, const int32_t* perm) { return r < n_inst ? perm[r] : r; }
__device__ __forceinline__ int map_col(int c, int n_inst, const int32_t* iperm) { return c < n_inst ? iperm[c] : c; }

__global__ void k_exec_lens(int32_t n_tot, int32_t n_inst, const int32_t* __restrict__ perm,
                            const int32_t* __restrict__ rp, int32_t* __restrict__ len) {
    int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n_tot) return;
    int s = src_row(static_cast<int>(r), n_inst, perm);
    len[r] = rp[s + 1] - rp[s];
}

// Execution-order netlist rows: each row copies its canonical row's
// entries (order kept) with columns renumbered and weights as float32.
// G lanes per row of at most kShortRow entries; one workgroup per longer
// row (k_exec_net_long).
constexpr int kShortRow = 64;

__device__ __forceinline__ int2 exec_entry(int32_t c, int64_t q, int n_inst, const int32_t* iperm) {
    return make_int2(map_col(c, n_inst, iperm), f_bits(static_cast<float>(static_cast<double>(q) * 0x1p-32)));
}

__global__ void __launch_bounds__(kBT) k_exec_net(int32_t n_tot, int32_t n_inst, const int32_t* __restrict__ perm,
                                                  const int32_t* __restrict__ iperm, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col, const int64_t* __restrict__ q,
                                                  const int32_t* __restrict__ xrp, int2* __restrict__ xent) {
    constexpr int G = 8;
    int64_t r = (static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x) / G;
    int l = threadIdx.x & (G - 1);
    if (r >= n_tot) return;
    int d = xrp[r], len = xrp[r + 1] - d;
    if (len > kShortRow) return;                           // group-uniform
    int a = rp[src_row(static_cast<int>(r), n_inst, perm)];
    for (int k = l; k < len; k += G) xent[d + k] = exec_entry(col[a + k], q[a + k], n_inst, iperm);
}

__global__ void __launch_bounds__(kBT) k_exec_net_long(const int32_t* __restrict__ rows, int32_t n_inst,
                                                       const int32_t* __restrict__ perm,
                                                       const int32_t* __restrict__ iperm,
                                                       const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                       const int64_t* __restrict__ q, const int32_t* __restrict__ xrp,
                                                       int2* __restrict__ xent) {
    const int r = rows[blockIdx.x];
    const int d = xrp[r], len = xrp[r + 1] - d;
    const int a = rp[src_row(r, n_inst, perm)];
    for (int k = threadIdx.x; k < len; k += kBT) xent[d + k] = exec_entry(col[a + k], q[a + k], n_inst, iperm);
}

__global__ void k_long_flags(int32_t n_tot, const int32_t* __restrict__ xrp, int32_t* __restrict__ flag) {
    int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r < n_tot) flag[r] = (xrp[r + 1] - xrp[r] > kShortRow) ? 1 : 0;
}

__global__ void k_exec_qdeg(int32_t n_tot, int32_t n_inst, const int32_t* __restrict__ perm,
                            const int64_t* __restrict__ qdeg, int64_t* __restrict__ xqdeg) {
    int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r < n_tot) xqdeg[r] = qdeg[src_row(static_cast<int>(r), n_inst, perm)];
}

}  // namespace

void set_layout(Graph& g, const float* pos, int32_t ncols, hipStream_t s) {
    const int32_t n = g.n_inst, N = g.n_tot;
    DevBuf<int32_t> key;
    key.ensure(static_cast<size_t>(n) + 1, s);
    const float side = static_cast<float>(1 << kGridBits);
    float sx = side / (g.nl.die[2] - g.nl.die[0]);
    float sy = side / (g.nl.die[3] - g.nl.die[1]);
    hipLaunchKernelGGL(k_layout_keys, dim3(grid_for(n, kBT)), dim3(kBT), 0, s, pos, ncols, n, g.nl.die[0],
                       g.nl.die[1], sx, sy, key.p);
    AHR_LAUNCHED("k_layout_keys");
    bucket_sort(g, key.p, n, 1 << (2 * kGridBits), g.perm, g.lay_start, s, false);   // every key >= 0
    key.release(s);
    g.iperm.ensure(static_cast<size_t>(n) + 1, s);
    hipLaunchKernelGGL(k_iperm, dim3(grid_for(n, kBT)), dim3(kBT), 0, s, g.perm.p, n, g.iperm.p);
    AHR_LAUNCHED("k_iperm");

    DevBuf<int32_t> len;
    len.ensure(static_cast<size_t>(N) + 1, s);
    hipLaunchKernelGGL(k_exec_lens, dim3(grid_for(N, kBT)), dim3(kBT), 0, s, N, n, g.perm.p, g.net_rp.p, len.p);
    AHR_LAUNCHED("k_exec_lens");
    g.xnet_rp.ensure(static_cast<size_t>(N) + 1, s);
    g.scan_tmp.ensure(scan_tmp_elems(N), s);
    scan_i32_to_i32(len.p, g.xnet_rp.p, N, g.scan_tmp.p, s);
    len.release(s);
    g.xnet_ent.ensure(static_cast<size_t>(g.nnz_net) + 1, s);
    g.xqdeg.ensure(static_cast<size_t>(N) + 1, s);
    if (g.nnz_net) {
        hipLaunchKernelGGL(k_exec_net, dim3(grid_for(static_cast<int64_t>(N) * 8, kBT)), dim3(kBT), 0, s, N, n,
                           g.perm.p, g.iperm.p, g.net_rp.p, g.net_col.p, g.net_q.p, g.xnet_rp.p, g.xnet_ent.p);
        AHR_LAUNCHED("k_exec_net");
        DevBuf<int32_t> flag, rank, rows;
        flag.ensure(static_cast<size_t>(N) + 1, s);
        rank.ensure(static_cast<size_t>(N) + 1, s);
        hipLaunchKernelGGL(k_long_flags, dim3(grid_for(N, kBT)), dim3(kBT), 0, s, N, g.xnet_rp.p, flag.p);
        AHR_LAUNCHED("k_long_flags");
        scan_i32_to_i32(flag.p, rank.p, N, g.scan_tmp.p, s);
        int32_t n_long = 0;
        read_scalars({rank.p + N}, &n_long, s);
        if (n_long) {
            rows.ensure(static_cast<size_t>(n_long) + 1, s);
            list_rows(flag.p, rank.p, N, rows.p, s);
            hipLaunchKernelGGL(k_exec_net_long, dim3(n_long), dim3(kBT), 0, s, rows.p, n, g.perm.p, g.iperm.p,
                               g.net_rp.p, g.net_col.p, g.net_q.p, g.xnet_rp.p, g.xnet_ent.p);
            AHR_LAUNCHED("k_exec_net_long");
        }
        flag.release(s);
        rank.release(s);
        rows.release(s);
    }
    hipLaunchKernelGGL(k_exec_qdeg, dim3(grid_for(N, kBT)), dim3(kBT), 0, s, N, n, g.perm.p, g.qdeg.p, g.xqdeg.p);
    AHR_LAUNCHED("k_exec_qdeg");
    g.has_layout = 1;
}

}  // namespace ahr
