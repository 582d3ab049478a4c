// Half-perimeter wirelength of every placement in a signal: per net and per
// (x, y) column pair, (max - min) of the pin x plus that of the pin y, pin
// position = instance position + pin offset, in float64.  Net totals are
// accumulated in a fixed order: a fixed grid of workgroups, each adding its
// nets in order, then one workgroup adding the workgroup partials in order.
#include "ahr_internal.hpp"
#include "device_util.hpp"

namespace ahr {

namespace {

constexpr int kBT = 256;
constexpr int kLanes = 8;           // lanes per small net
constexpr int kSmallGrid = 8192;    // workgroups of the small-net pass (enough nets in flight
                                    // to hide the two dependent loads of each)
constexpr int kBigGrid = 256;       // workgroups of the big-net pass
constexpr int kMaxPairs = 4;

// Workgroup partials (fixed size; shared by every call on a device).
__device__ double g_hpwl_partial[(kSmallGrid + kBigGrid) * kMaxPairs];

template <int P>
__device__ __forceinline__ void pin_bounds(const float* pos, int ncols, const int32_t* pin_node, const float* pin_off,
                                           int p, double* lo, double* hi) {
    int v = pin_node[p];
    double ox = pin_off[2 * p], oy = pin_off[2 * p + 1];
    const float* g = pos + static_cast<int64_t>(v) * ncols;
#pragma unroll
    for (int c = 0; c < 2 * P; ++c) {
        double x = static_cast<double>(g[c]) + ((c & 1) ? oy : ox);
        lo[c] = x < lo[c] ? x : lo[c];
        hi[c] = x > hi[c] ? x : hi[c];
    }
}

// Nets with at most a wave's worth of pins: kLanes lanes per net.
template <int P>
__global__ void __launch_bounds__(kBT) k_hpwl_small(const float* __restrict__ pos, int ncols,
                                                    const int32_t* __restrict__ net_ptr, int32_t n_nets,
                                                    const int32_t* __restrict__ pin_node,
                                                    const float* __restrict__ pin_off) {
    __shared__ double red[kBT / kWave];
    const int l = threadIdx.x & (kLanes - 1);
    const int64_t groups = static_cast<int64_t>(kSmallGrid) * (kBT / kLanes);
    double tot[P];
#pragma unroll
    for (int c = 0; c < P; ++c) tot[c] = 0;
    for (int64_t e = (static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x) / kLanes; e < n_nets; e += groups) {
        int p0 = net_ptr[e], p1 = net_ptr[e + 1];
        if (p1 - p0 > kWave || p1 - p0 < 1) continue;   // group-uniform
        double lo[2 * P], hi[2 * P];
#pragma unroll
        for (int c = 0; c < 2 * P; ++c) {
            lo[c] = 1e300;
            hi[c] = -1e300;
        }
        for (int p = p0 + l; p < p1; p += kLanes) pin_bounds<P>(pos, ncols, pin_node, pin_off, p, lo, hi);
#pragma unroll
        for (int o = kLanes / 2; o > 0; o >>= 1) {
#pragma unroll
            for (int c = 0; c < 2 * P; ++c) {
                double a = __shfl_xor(lo[c], o), b = __shfl_xor(hi[c], o);
                lo[c] = a < lo[c] ? a : lo[c];
                hi[c] = b > hi[c] ? b : hi[c];
            }
        }
        if (l == 0) {
#pragma unroll
            for (int c = 0; c < P; ++c) tot[c] += (hi[2 * c] - lo[2 * c]) + (hi[2 * c + 1] - lo[2 * c + 1]);
        }
    }
#pragma unroll
    for (int c = 0; c < P; ++c) {
        double s = block_sum_f64<kBT>(tot[c], red);
        if (threadIdx.x == 0) g_hpwl_partial[blockIdx.x * kMaxPairs + c] = s;
    }
}

// Nets with more pins: one workgroup per net (grid-stride over the list).
template <int P>
__global__ void __launch_bounds__(kBT) k_hpwl_big(const float* __restrict__ pos, int ncols,
                                                  const int32_t* __restrict__ net_ptr,
                                                  const int32_t* __restrict__ big, int32_t n_big,
                                                  const int32_t* __restrict__ pin_node,
                                                  const float* __restrict__ pin_off) {
    __shared__ double red[2 * 2 * P][kBT / kWave];
    double tot[P];
#pragma unroll
    for (int c = 0; c < P; ++c) tot[c] = 0;
    for (int k = blockIdx.x; k < n_big; k += kBigGrid) {
        int e = big[k];
        int p0 = net_ptr[e], p1 = net_ptr[e + 1];
        double lo[2 * P], hi[2 * P];
#pragma unroll
        for (int c = 0; c < 2 * P; ++c) {
            lo[c] = 1e300;
            hi[c] = -1e300;
        }
        for (int p = p0 + threadIdx.x; p < p1; p += kBT) pin_bounds<P>(pos, ncols, pin_node, pin_off, p, lo, hi);
#pragma unroll
        for (int c = 0; c < 2 * P; ++c) {
            lo[c] = -wave_max(-lo[c]);
            hi[c] = wave_max(hi[c]);
        }
        __syncthreads();
        if (lane_id() == 0) {
#pragma unroll
            for (int c = 0; c < 2 * P; ++c) {
                red[2 * c][wave_id()] = lo[c];
                red[2 * c + 1][wave_id()] = hi[c];
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
#pragma unroll
            for (int c = 0; c < P; ++c) {
                double h = 0;
#pragma unroll
                for (int d = 0; d < 2; ++d) {
                    double a = red[2 * (2 * c + d)][0], b = red[2 * (2 * c + d) + 1][0];
                    for (int w = 1; w < kBT / kWave; ++w) {
                        a = red[2 * (2 * c + d)][w] < a ? red[2 * (2 * c + d)][w] : a;
                        b = red[2 * (2 * c + d) + 1][w] > b ? red[2 * (2 * c + d) + 1][w] : b;
                    }
                    h += b - a;
                }
                tot[c] += h;
            }
        }
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < P; ++c) g_hpwl_partial[(kSmallGrid + blockIdx.x) * kMaxPairs + c] = tot[c];
    }
}

// The workgroup partials in a fixed order: thread t adds partials t,
// t + kFinalBT, ... (all loaded at once), then a fixed block reduction.
constexpr int kFinalBT = 1024;
constexpr int kFinalPer = (kSmallGrid + kBigGrid + kFinalBT - 1) / kFinalBT;

__global__ void __launch_bounds__(kFinalBT) k_hpwl_final(int npairs, double* __restrict__ out) {
    __shared__ double red[kFinalBT / kWave];
    constexpr int nparts = kSmallGrid + kBigGrid;
    for (int c = 0; c < npairs; ++c) {
        double v[kFinalPer];
#pragma unroll
        for (int u = 0; u < kFinalPer; ++u) {
            const int b = static_cast<int>(threadIdx.x) + u * kFinalBT;
            v[u] = g_hpwl_partial[(b < nparts ? b : nparts - 1) * kMaxPairs + c];
        }
        double s = 0;
#pragma unroll
        for (int u = 0; u < kFinalPer; ++u) s += static_cast<int>(threadIdx.x) + u * kFinalBT < nparts ? v[u] : 0.0;
        s = block_sum_f64<kFinalBT>(s, red);
        if (threadIdx.x == 0) out[c] = s;
    }
}

template <int P>
void hpwl_p(const Graph& g, const float* pos, int32_t ncols, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_hpwl_small<P>, dim3(kSmallGrid), dim3(kBT), 0, s, pos, ncols, g.nl.net_ptr, g.nl.n_nets,
                       g.nl.pin_node, g.nl.pin_off);
    AHR_LAUNCHED("k_hpwl_small");
    hipLaunchKernelGGL(k_hpwl_big<P>, dim3(kBigGrid), dim3(kBT), 0, s, pos, ncols, g.nl.net_ptr, g.big_nets.p,
                       g.n_big_nets, g.nl.pin_node, g.nl.pin_off);
    AHR_LAUNCHED("k_hpwl_big");
    hipLaunchKernelGGL(k_hpwl_final, dim3(1), dim3(kFinalBT), 0, s, P, out);
    AHR_LAUNCHED("k_hpwl_final");
}

}  // namespace

void run_hpwl(const Graph& g, const float* pos, int32_t ncols, double* out, hipStream_t s) {
    ProfScope ps(kStageHpwl, s);
    switch (ncols) {
        case 2: hpwl_p<1>(g, pos, ncols, out, s); break;
        case 4: hpwl_p<2>(g, pos, ncols, out, s); break;
        case 8: hpwl_p<4>(g, pos, ncols, out, s); break;
        default: throw Error{AHR_EUNSUPPORTED, "hpwl needs ncols of 2, 4 or 8"};
    }
}

}  // namespace ahr
