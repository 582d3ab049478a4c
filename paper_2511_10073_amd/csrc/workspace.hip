// The device workspace a graph needs when the caller provides its memory
// (ahr_graph_workspace_size): an upper bound on the bytes the graph holds at
// once, from the netlist's exact sizes (one counting pass over the nets and
// pins on the device) and bounds on what the placement decides.
//
// Terms (bytes), with N instances, P pins, E nets, B bins, C columns:
//   raw  netlist entries before merging, sum over nets of p (p - 1) for a
//        clique and 2p for a star: the build holds each as a 16-byte record,
//        its column and weight (12 bytes) and a sort key (8), and keeps the
//        merged copy and the execution-order copy (8);
//   H    hint entries: twice the (cell, macro) pairs, at most 4 per movable
//        standard cell (a point lies in at most four footprints that do not
//        overlap), plus twice the cells times the detection window's slots;
//        each an 8-byte entry, with the sparsification's compaction copy;
//   B    per bin: densities, phi, the macros' kept areas, bin lists;
//   rows N + macro pin nodes + star nodes + macro and bin virtual nodes:
//        row pointers, layout, degrees, scales, hop coefficients, row
//        classes and the filter's signal buffers (about 11 C floats a row);
//   per instance, pin and net: the netlist order's level arrays, the hint
//        build's per-cell arrays (with the pruning's kept-slot mask), the
//        refinement's three placements, pin maps and net lists.
// A 25 % margin covers the sub-allocator's fragmentation.
#include <cmath>

#include "ahr_internal.hpp"
#include "device_util.hpp"

namespace ahr {

namespace {

constexpr int kBT = 256;

// counts[0] raw netlist entries, [1] star nets, [2] pins on fixed macros
// (when they are expanded), [3] macros, [4] movable standard cells
__global__ void __launch_bounds__(kBT) k_ws_counts(const int32_t* __restrict__ net_ptr, int32_t n_nets,
                                                   const int32_t* __restrict__ pin_node, int32_t n_pins,
                                                   const uint8_t* __restrict__ flags, int32_t n_inst,
                                                   int32_t clique_max, int expand, unsigned long long* counts) {
    __shared__ int64_t red[kBT / kWave];
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x;
    int64_t raw = 0, star = 0, mpin = 0, mac = 0, std_cells = 0;
    if (i < n_nets) {
        const int64_t p = net_ptr[i + 1] - net_ptr[i];
        if (p >= 2) {
            if (p <= clique_max) {
                raw = p * (p - 1);
            } else {
                raw = 2 * p;
                star = 1;
            }
        }
    }
    if (i < n_pins && expand) {
        const uint8_t f = flags[pin_node[i]];
        mpin = (f & AHR_NODE_FIXED) && (f & AHR_NODE_MACRO) ? 1 : 0;
    }
    if (i < n_inst) {
        const uint8_t f = flags[i];
        mac = (f & AHR_NODE_MACRO) ? 1 : 0;
        std_cells = f == 0 ? 1 : 0;
    }
    const int64_t v[5] = {raw, star, mpin, mac, std_cells};
    for (int k = 0; k < 5; ++k) {
        const int64_t s = block_sum_i64<kBT>(v[k], red);
        if (threadIdx.x == 0 && s) atomicAdd(&counts[k], static_cast<unsigned long long>(s));
    }
}

__global__ void k_zero5(unsigned long long* c) {
    if (threadIdx.x < 5) c[threadIdx.x] = 0ull;
}

int half_window(float ratio, int nb) {
    const float f = std::floor(ratio * static_cast<float>(nb));
    const int n = f < 1.f ? 1 : static_cast<int>(f);
    return n / 2;
}

}  // namespace

size_t graph_workspace_bytes(const ahr_netlist& nl, const ahr_hint_params& hp, int32_t ncols, hipStream_t s) {
    const int64_t N = nl.n_inst, P = nl.n_pins, E = nl.n_nets;
    const int64_t n = std::max<int64_t>(std::max<int64_t>(N, P), E);
    DevBuf<unsigned long long> c;
    c.ensure(5, s);
    hipLaunchKernelGGL(k_zero5, dim3(1), dim3(64), 0, s, c.p);
    AHR_LAUNCHED("k_zero5");
    hipLaunchKernelGGL(k_ws_counts, dim3(grid_for(n, kBT)), dim3(kBT), 0, s, nl.net_ptr, nl.n_nets, nl.pin_node,
                       nl.n_pins, nl.node_flags, nl.n_inst, hp.clique_max, (hp.flags & AHR_EXPAND_MACRO_PINS) ? 1 : 0,
                       c.p);
    AHR_LAUNCHED("k_ws_counts");
    unsigned long long h[5];
    AHR_HIP(hipMemcpyAsync(h, c.p, sizeof h, hipMemcpyDeviceToHost, s));
    AHR_HIP(hipStreamSynchronize(s));
    c.release(s);
    const double raw = static_cast<double>(h[0]), stars = static_cast<double>(h[1]);
    const double mpin = static_cast<double>(h[2]), macros = static_cast<double>(h[3]);
    const double cells = static_cast<double>(h[4]);
    const bool mh = hp.flags & AHR_MACRO_HINTS, bh = hp.flags & AHR_BIN_HINTS;
    const double B = bh ? static_cast<double>(hp.nbx) * hp.nby : 0.0;
    const double wslots = bh ? static_cast<double>(2 * half_window(hp.detection_ratio, hp.nbx) + 1) *
                                   (2 * half_window(hp.detection_ratio, hp.nby) + 1)
                             : 0.0;
    const double H = 2 * ((mh ? 4 * cells : 0.0) + (bh ? cells * wslots : 0.0));
    const double rows = static_cast<double>(N) + mpin + stars + (mh ? macros : 0.0) + B;
    const double C = ncols > 0 ? ncols : 8;
    const double bytes = 48 * raw + 40 * H + (176 + 44 * C) * rows + (296 + 12 * C) * static_cast<double>(N) +
                         64 * static_cast<double>(P) + 48 * static_cast<double>(E) + 16 * B * wslots + 40 * B;
    return static_cast<size_t>(1.25 * bytes) + (size_t(32) << 20);
}

size_t graph_workspace_floor(const ahr_netlist& nl, int32_t ncols) {
    // arrays every graph holds whatever the netlist's contents: per-pin node
    // maps, per-row offsets and lengths of the instance rows, per-instance
    // refinement placements
    const size_t C = ncols > 0 ? static_cast<size_t>(ncols) : 8;
    return static_cast<size_t>(nl.n_pins) * 4 + static_cast<size_t>(nl.n_inst) * (12 + 12 * C) +
           static_cast<size_t>(nl.n_nets) * 4;
}

}  // namespace ahr
