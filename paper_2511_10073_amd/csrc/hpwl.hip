// Half-perimeter wirelength of every placement in a signal: per net and per
// (x, y) column pair, (max - min) of the pin x plus that of the pin y, pin
// position = instance position + pin offset, in float64.
//
// Each workgroup owns one contiguous range of nets.  Nets with at most a
// wave's worth of pins take kLanes lanes each; the rest of the range's nets
// are then summed one after another by the whole workgroup.  Workgroup
// totals go to a partial-sum buffer, which one workgroup adds in a fixed
// order, so the result is deterministic and no list of the big nets is
// needed: the pass reads the netlist arrays alone.
//
// ahr_hpwl draws the partial-sum buffer from the library's stream-ordered
// pool for each call, so calls on different streams share no memory.
#include "ahr_internal.hpp"
#include "device_util.hpp"

namespace ahr {

namespace {

constexpr int kBT = 256;
constexpr int kLanes = 8;           // lanes per small net
constexpr int kGroups = kBT / kLanes;
constexpr int kMaxGrid = 8192;      // workgroups (enough nets in flight to hide the two dependent loads of each)
constexpr int kNetsPerWg = 256;     // fewer nets per workgroup only below kMaxGrid workgroups
constexpr int kMaxPairs = 4;        // ncols <= 8
constexpr size_t kPartialElems = static_cast<size_t>(kMaxGrid) * kMaxPairs;

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

template <int P>
__global__ void __launch_bounds__(kBT) k_hpwl(const float* __restrict__ pos, int ncols,
                                              const int32_t* __restrict__ net_ptr, int32_t n_nets, int32_t per,
                                              const int32_t* __restrict__ pin_node, const float* __restrict__ pin_off,
                                              double* __restrict__ partial) {
    __shared__ double red[kBT / kWave];
    __shared__ double ext[2 * 2 * P][kBT / kWave];
    __shared__ unsigned long long big_mask[kBT / kWave];
    const int64_t lo_net = static_cast<int64_t>(blockIdx.x) * per;
    const int64_t hi_net = lo_net + per < n_nets ? lo_net + per : n_nets;
    const int l = threadIdx.x & (kLanes - 1);
    double tot[P];
#pragma unroll
    for (int c = 0; c < P; ++c) tot[c] = 0;

    // nets of at most kWave pins: kLanes lanes each
    for (int64_t e = lo_net + threadIdx.x / kLanes; e < hi_net; e += kGroups) {
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

    // the range's bigger nets, in net order, by the whole workgroup
    for (int64_t c0 = lo_net; c0 < hi_net; c0 += kBT) {
        const int64_t e = c0 + threadIdx.x;
        const bool big = e < hi_net && net_ptr[e + 1] - net_ptr[e] > kWave;
        const unsigned long long m = __ballot(big);
        __syncthreads();
        if (lane_id() == 0) big_mask[wave_id()] = m;
        __syncthreads();
        for (int w = 0; w < kBT / kWave; ++w) {
            unsigned long long mm = big_mask[w];          // uniform over the workgroup
            while (mm) {
                const int b = __ffsll(static_cast<long long>(mm)) - 1;
                mm &= mm - 1;
                const int64_t net = c0 + w * kWave + b;
                const int p0 = net_ptr[net], p1 = net_ptr[net + 1];
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
                        ext[2 * c][wave_id()] = lo[c];
                        ext[2 * c + 1][wave_id()] = hi[c];
                    }
                }
                __syncthreads();
                if (threadIdx.x == 0) {
#pragma unroll
                    for (int c = 0; c < P; ++c) {
                        double h = 0;
#pragma unroll
                        for (int d = 0; d < 2; ++d) {
                            double a = ext[2 * (2 * c + d)][0], bb = ext[2 * (2 * c + d) + 1][0];
                            for (int u = 1; u < kBT / kWave; ++u) {
                                a = ext[2 * (2 * c + d)][u] < a ? ext[2 * (2 * c + d)][u] : a;
                                bb = ext[2 * (2 * c + d) + 1][u] > bb ? ext[2 * (2 * c + d) + 1][u] : bb;
                            }
                            h += bb - a;
                        }
                        tot[c] += h;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < P; ++c) {
        double s = block_sum_f64<kBT>(tot[c], red);
        if (threadIdx.x == 0) partial[static_cast<int64_t>(blockIdx.x) * kMaxPairs + c] = s;
    }
}

// The workgroup partials in a fixed order: thread t adds partials t,
// t + kFinalBT, ... (all loaded at once), then a fixed block reduction.
constexpr int kFinalBT = 1024;
constexpr int kFinalPer = (kMaxGrid + kFinalBT - 1) / kFinalBT;

__global__ void __launch_bounds__(kFinalBT) k_hpwl_final(const double* __restrict__ partial, int nparts, int npairs,
                                                         double* __restrict__ out) {
    __shared__ double red[kFinalBT / kWave];
    for (int c = 0; c < npairs; ++c) {
        double v[kFinalPer];
#pragma unroll
        for (int u = 0; u < kFinalPer; ++u) {
            const int b = static_cast<int>(threadIdx.x) + u * kFinalBT;
            v[u] = partial[(b < nparts ? b : nparts - 1) * kMaxPairs + c];
        }
        double s = 0;
#pragma unroll
        for (int u = 0; u < kFinalPer; ++u) s += static_cast<int>(threadIdx.x) + u * kFinalBT < nparts ? v[u] : 0.0;
        s = block_sum_f64<kFinalBT>(s, red);
        if (threadIdx.x == 0) out[c] = s;
    }
}

int hpwl_grid(int32_t n_nets) {
    int64_t g = (static_cast<int64_t>(n_nets) + kNetsPerWg - 1) / kNetsPerWg;
    return static_cast<int>(g < 1 ? 1 : (g > kMaxGrid ? kMaxGrid : g));
}

template <int P>
void hpwl_p(const ahr_netlist& nl, const float* pos, int32_t ncols, double* out, double* partial, hipStream_t s) {
    const int grid = hpwl_grid(nl.n_nets);
    const int32_t per = static_cast<int32_t>((static_cast<int64_t>(nl.n_nets) + grid - 1) / grid);
    hipLaunchKernelGGL(k_hpwl<P>, dim3(grid), dim3(kBT), 0, s, pos, ncols, nl.net_ptr, nl.n_nets, per, nl.pin_node,
                       nl.pin_off, partial);
    AHR_LAUNCHED("k_hpwl");
    hipLaunchKernelGGL(k_hpwl_final, dim3(1), dim3(kFinalBT), 0, s, partial, grid, P, out);
    AHR_LAUNCHED("k_hpwl_final");
}

}  // namespace

void hpwl_launch(const ahr_netlist& nl, const float* pos, int32_t ncols, double* out, double* partial,
                 hipStream_t s) {
    switch (ncols) {
        case 2: hpwl_p<1>(nl, pos, ncols, out, partial, s); break;
        case 4: hpwl_p<2>(nl, pos, ncols, out, partial, s); break;
        case 8: hpwl_p<4>(nl, pos, ncols, out, partial, s); break;
        default: throw Error{AHR_EUNSUPPORTED, "hpwl needs ncols of 2, 4 or 8"};
    }
}

size_t hpwl_partial_elems() { return kPartialElems; }

void run_hpwl(const ahr_netlist& nl, const float* pos, int32_t ncols, double* out, hipStream_t s) {
    ProfScope ps(kStageHpwl, s);
    DevBuf<double> partial;
    partial.ensure(static_cast<size_t>(hpwl_grid(nl.n_nets)) * kMaxPairs, s);
    hpwl_launch(nl, pos, ncols, out, partial.p, s);
    partial.release(s);
}

}  // namespace ahr
