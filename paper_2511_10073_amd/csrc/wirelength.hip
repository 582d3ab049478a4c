// Weighted-average (WA) wirelength and its gradient (Section II-B of the
// paper, "Wirelength model"): for each net and axis the exponentially
// weighted means of the pin coordinates with weights exp(+x/gamma) (smooth
// maximum) and exp(-x/gamma) (smooth minimum); W sums their differences over
// nets and both axes.  This is the wirelength term of the electrostatic
// global placer that consumes the initializer's placement.
//
// Numbers: float64 throughout; each weight is taken relative to the net's
// extreme coordinate (exp((x - max)/gamma), exp((min - x)/gamma)), which
// cancels in every ratio.  Gradient of pin i:
//   p+_i (1 + (x_i - xbar+)/gamma) - p-_i (1 - (x_i - xbar-)/gamma),
// p+-_i the pin's normalised weight.  An instance's gradient is the sum over
// its pins, added in int64 fixed point (2^-40 units), so the order in which
// the node pass meets the pins does not change the result.
//
// Layout: an index built once per netlist (ahr_wl_create) lists every
// instance's pins (node_ptr / node_pins) and gives each pin its position in
// that list (pin_slot).  One call is three kernels: the net pass (net totals
// into workgroup partials; per-pin gradients written at the pin's position,
// so every instance's pins lie together in a [pins][ncols] float64 buffer),
// the node pass (one thread per instance, contiguous reads), and the
// fixed-order reduction of the partials.  Nets of at most 8 pins keep one
// pin per lane in registers (one gather); larger ones loop over their pins.
#include <cmath>

#include "ahr_internal.hpp"
#include "device_util.hpp"

namespace ahr {

namespace {

constexpr int kBT = 256;
constexpr int kLanes = 8;
constexpr int kGroups = kBT / kLanes;
constexpr int kMaxGrid = 8192;
constexpr int kNetsPerWg = 256;
constexpr int kMaxPairs = 4;
constexpr double kFix = 1099511627776.0;          // 2^40
constexpr double kUnfix = 1.0 / 1099511627776.0;

struct WlIndex {
    ahr_netlist nl;
    DevBuf<int32_t> node_ptr;     // [n_inst + 1]
    DevBuf<int32_t> node_pins;    // [n_pins] pins of each instance (order within an instance unspecified)
    DevBuf<int32_t> pin_slot;     // [n_pins] position of each pin in node_pins
    int device = 0;
    mutable hipStream_t work_stream = nullptr;
    mutable int stream_uses = 0;
    void use_stream(hipStream_t s) const {
        if (stream_uses == 0) {
            work_stream = s;
            stream_uses = 1;
        } else if (s != work_stream) {
            stream_uses = 2;
        }
    }
    ~WlIndex() {
        hipStream_t s = stream_uses == 1 ? work_stream : nullptr;
        if (stream_uses > 1) (void)hipDeviceSynchronize();
        node_ptr.release(s);
        node_pins.release(s);
        pin_slot.release(s);
    }
};

__global__ void k_pin_slots(const int32_t* __restrict__ pin_node, int32_t n_pins, int32_t* __restrict__ cnt,
                            int32_t* __restrict__ slot) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p < n_pins) slot[p] = atomicAdd(&cnt[pin_node[p]], 1);
}

__global__ void k_pin_scatter(const int32_t* __restrict__ pin_node, int32_t n_pins, int32_t* __restrict__ slot,
                              const int32_t* __restrict__ node_ptr, int32_t* __restrict__ node_pins) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p < n_pins) {
        const int32_t k = node_ptr[pin_node[p]] + slot[p];
        node_pins[k] = static_cast<int32_t>(p);
        slot[p] = k;          // from here on: the pin's position in node_pins
    }
}

// Coordinate of pin p in column c: instance position + pin offset (x or y).
__device__ __forceinline__ double pin_coord(const float* pos, int ncols, const int32_t* pin_node, const float* pin_off,
                                            int p, int c) {
    return static_cast<double>(pos[static_cast<int64_t>(pin_node[p]) * ncols + c]) +
           static_cast<double>(pin_off[2 * p + (c & 1)]);
}

// Per-net WA over the column range [0, 2P): the caller reduces the lane
// partials (RED: lanes of one group or a whole workgroup) between passes.
template <int P>
struct NetAcc {
    double hi[2 * P], lo[2 * P];      // extremes
    double sp[2 * P], tp[2 * P];      // sum exp((x-hi)/g), sum x exp((x-hi)/g)
    double sm[2 * P], tm[2 * P];      // sum exp((lo-x)/g), sum x exp((lo-x)/g)
};

template <int P>
__device__ __forceinline__ void acc_bounds(NetAcc<P>& a, const float* pos, int ncols, const int32_t* pin_node,
                                           const float* pin_off, int p) {
#pragma unroll
    for (int c = 0; c < 2 * P; ++c) {
        double x = pin_coord(pos, ncols, pin_node, pin_off, p, c);
        a.hi[c] = x > a.hi[c] ? x : a.hi[c];
        a.lo[c] = x < a.lo[c] ? x : a.lo[c];
    }
}

template <int P>
__device__ __forceinline__ void acc_sums(NetAcc<P>& a, const float* pos, int ncols, const int32_t* pin_node,
                                         const float* pin_off, int p, double inv_g) {
#pragma unroll
    for (int c = 0; c < 2 * P; ++c) {
        double x = pin_coord(pos, ncols, pin_node, pin_off, p, c);
        double ep = exp((x - a.hi[c]) * inv_g), em = exp((a.lo[c] - x) * inv_g);
        a.sp[c] += ep;
        a.tp[c] += x * ep;
        a.sm[c] += em;
        a.tm[c] += x * em;
    }
}

template <int P>
__device__ __forceinline__ void pin_grads(const NetAcc<P>& a, const float* pos, int ncols, const int32_t* pin_node,
                                          const float* pin_off, int p, double inv_g, double* pin_g,
                                          const int32_t* pin_slot) {
    const int64_t k = pin_slot[p];
#pragma unroll
    for (int c = 0; c < 2 * P; ++c) {
        double x = pin_coord(pos, ncols, pin_node, pin_off, p, c);
        double xp = a.tp[c] / a.sp[c], xm = a.tm[c] / a.sm[c];
        double pp = exp((x - a.hi[c]) * inv_g) / a.sp[c], pm = exp((a.lo[c] - x) * inv_g) / a.sm[c];
        pin_g[k * ncols + c] = pp * (1.0 + (x - xp) * inv_g) - pm * (1.0 - (x - xm) * inv_g);
    }
}

template <int P>
__device__ __forceinline__ void init_acc(NetAcc<P>& a) {
#pragma unroll
    for (int c = 0; c < 2 * P; ++c) {
        a.hi[c] = -1e300;
        a.lo[c] = 1e300;
        a.sp[c] = a.tp[c] = a.sm[c] = a.tm[c] = 0.0;
    }
}

template <int P>
__device__ __forceinline__ double net_wa(const NetAcc<P>& a, int pair) {
    double w = 0;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        const int c = 2 * pair + d;
        w += a.tp[c] / a.sp[c] - a.tm[c] / a.sm[c];
    }
    return w;
}

// Reduction of the kLanes lanes of a group (shuffles, fixed order).
template <int P>
__device__ __forceinline__ void group_bounds(NetAcc<P>& a) {
#pragma unroll
    for (int o = kLanes / 2; o > 0; o >>= 1) {
#pragma unroll
        for (int c = 0; c < 2 * P; ++c) {
            double h = __shfl_xor(a.hi[c], o), l = __shfl_xor(a.lo[c], o);
            a.hi[c] = h > a.hi[c] ? h : a.hi[c];
            a.lo[c] = l < a.lo[c] ? l : a.lo[c];
        }
    }
}

template <int P>
__device__ __forceinline__ void group_sums(NetAcc<P>& a) {
#pragma unroll
    for (int o = kLanes / 2; o > 0; o >>= 1) {
#pragma unroll
        for (int c = 0; c < 2 * P; ++c) {
            a.sp[c] += __shfl_xor(a.sp[c], o);
            a.tp[c] += __shfl_xor(a.tp[c], o);
            a.sm[c] += __shfl_xor(a.sm[c], o);
            a.tm[c] += __shfl_xor(a.tm[c], o);
        }
    }
}

// Whole-workgroup reductions of one net's values (every thread gets them);
// red holds kBT / kWave doubles and is reused after a barrier.
__device__ __forceinline__ double block_max_f64(double v, double* red) {
    v = wave_max(v);
    __syncthreads();
    if (lane_id() == 0) red[wave_id()] = v;
    __syncthreads();
    double t = red[0];
#pragma unroll
    for (int w = 1; w < kBT / kWave; ++w) t = red[w] > t ? red[w] : t;
    return t;
}

template <int P>
__global__ void __launch_bounds__(kBT) k_wa_nets(const float* __restrict__ pos, int ncols,
                                                 const int32_t* __restrict__ net_ptr, int32_t n_nets, int32_t per,
                                                 const int32_t* __restrict__ pin_node,
                                                 const float* __restrict__ pin_off, double inv_g,
                                                 double* __restrict__ partial, double* __restrict__ pin_g,
                                                 const int32_t* __restrict__ pin_slot) {
    __shared__ double red[kBT / kWave];
    __shared__ unsigned long long big_mask[kBT / kWave];
    const int64_t lo_net = static_cast<int64_t>(blockIdx.x) * per;
    const int64_t hi_net = lo_net + per < n_nets ? lo_net + per : n_nets;
    const int l = threadIdx.x & (kLanes - 1);
    double tot[P];
#pragma unroll
    for (int c = 0; c < P; ++c) tot[c] = 0;

    for (int64_t e = lo_net + threadIdx.x / kLanes; e < hi_net; e += kGroups) {
        const int p0 = net_ptr[e], p1 = net_ptr[e + 1];
        if (p1 - p0 > kWave || p1 - p0 < 1) continue;   // group-uniform
        if (p1 - p0 <= kLanes) {
            // at most one pin per lane: its coordinates and weights stay in
            // registers (one gather, two exponentials per column)
            const bool has = p0 + l < p1;
            const int p = has ? p0 + l : p0;
            double x[2 * P], hi[2 * P], lo[2 * P];
#pragma unroll
            for (int c = 0; c < 2 * P; ++c) {
                x[c] = pin_coord(pos, ncols, pin_node, pin_off, p, c);
                hi[c] = has ? x[c] : -1e300;
                lo[c] = has ? x[c] : 1e300;
            }
#pragma unroll
            for (int o = kLanes / 2; o > 0; o >>= 1) {
#pragma unroll
                for (int c = 0; c < 2 * P; ++c) {
                    const double h2 = __shfl_xor(hi[c], o), l2 = __shfl_xor(lo[c], o);
                    hi[c] = h2 > hi[c] ? h2 : hi[c];
                    lo[c] = l2 < lo[c] ? l2 : lo[c];
                }
            }
            double ep[2 * P], em[2 * P], sp[2 * P], tp[2 * P], sm[2 * P], tm[2 * P];
#pragma unroll
            for (int c = 0; c < 2 * P; ++c) {
                ep[c] = has ? exp((x[c] - hi[c]) * inv_g) : 0.0;
                em[c] = has ? exp((lo[c] - x[c]) * inv_g) : 0.0;
                sp[c] = ep[c];
                tp[c] = x[c] * ep[c];
                sm[c] = em[c];
                tm[c] = x[c] * em[c];
            }
#pragma unroll
            for (int o = kLanes / 2; o > 0; o >>= 1) {
#pragma unroll
                for (int c = 0; c < 2 * P; ++c) {
                    sp[c] += __shfl_xor(sp[c], o);
                    tp[c] += __shfl_xor(tp[c], o);
                    sm[c] += __shfl_xor(sm[c], o);
                    tm[c] += __shfl_xor(tm[c], o);
                }
            }
            if (pin_g && has) {
                const int64_t k = pin_slot[p];
#pragma unroll
                for (int c = 0; c < 2 * P; ++c) {
                    const double xp = tp[c] / sp[c], xm = tm[c] / sm[c];
                    pin_g[k * ncols + c] =
                        ep[c] / sp[c] * (1.0 + (x[c] - xp) * inv_g) - em[c] / sm[c] * (1.0 - (x[c] - xm) * inv_g);
                }
            }
            if (l == 0) {
#pragma unroll
                for (int c = 0; c < P; ++c)
                    tot[c] += (tp[2 * c] / sp[2 * c] - tm[2 * c] / sm[2 * c]) +
                              (tp[2 * c + 1] / sp[2 * c + 1] - tm[2 * c + 1] / sm[2 * c + 1]);
            }
            continue;
        }
        NetAcc<P> a;
        init_acc(a);
        for (int p = p0 + l; p < p1; p += kLanes) acc_bounds<P>(a, pos, ncols, pin_node, pin_off, p);
        group_bounds<P>(a);
        for (int p = p0 + l; p < p1; p += kLanes) acc_sums<P>(a, pos, ncols, pin_node, pin_off, p, inv_g);
        group_sums<P>(a);
        if (pin_g)
            for (int p = p0 + l; p < p1; p += kLanes) pin_grads<P>(a, pos, ncols, pin_node, pin_off, p, inv_g, pin_g, pin_slot);
        if (l == 0) {
#pragma unroll
            for (int c = 0; c < P; ++c) tot[c] += net_wa<P>(a, c);
        }
    }

    // the range's nets above kWave pins, one after another, by the whole workgroup
    for (int64_t c0 = lo_net; c0 < hi_net; c0 += kBT) {
        const int64_t e = c0 + threadIdx.x;
        const bool big = e < hi_net && net_ptr[e + 1] - net_ptr[e] > kWave;
        const unsigned long long m = __ballot(big);
        __syncthreads();
        if (lane_id() == 0) big_mask[wave_id()] = m;
        __syncthreads();
        for (int w = 0; w < kBT / kWave; ++w) {
            unsigned long long mm = big_mask[w];
            while (mm) {
                const int b = __ffsll(static_cast<long long>(mm)) - 1;
                mm &= mm - 1;
                const int64_t net = c0 + w * kWave + b;
                const int p0 = net_ptr[net], p1 = net_ptr[net + 1];
                NetAcc<P> a;
                init_acc(a);
                for (int p = p0 + threadIdx.x; p < p1; p += kBT) acc_bounds<P>(a, pos, ncols, pin_node, pin_off, p);
#pragma unroll
                for (int c = 0; c < 2 * P; ++c) {
                    a.hi[c] = block_max_f64(a.hi[c], red);
                    a.lo[c] = -block_max_f64(-a.lo[c], red);
                }
                for (int p = p0 + threadIdx.x; p < p1; p += kBT) acc_sums<P>(a, pos, ncols, pin_node, pin_off, p, inv_g);
#pragma unroll
                for (int c = 0; c < 2 * P; ++c) {
                    a.sp[c] = block_sum_f64<kBT>(a.sp[c], red);
                    a.tp[c] = block_sum_f64<kBT>(a.tp[c], red);
                    a.sm[c] = block_sum_f64<kBT>(a.sm[c], red);
                    a.tm[c] = block_sum_f64<kBT>(a.tm[c], red);
                }
                if (pin_g)
                    for (int p = p0 + threadIdx.x; p < p1; p += kBT)
                        pin_grads<P>(a, pos, ncols, pin_node, pin_off, p, inv_g, pin_g, pin_slot);
                if (threadIdx.x == 0) {
#pragma unroll
                    for (int c = 0; c < P; ++c) tot[c] += net_wa<P>(a, c);
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

// Gradient of every instance: the exact (int64, 2^-40 units) sum of its
// pins' gradients, rounded once to float32.
template <int C>
__global__ void __launch_bounds__(kBT) k_wa_nodes(const int32_t* __restrict__ node_ptr,
                                                  const double* __restrict__ pin_g, int32_t n_inst,
                                                  float* __restrict__ grad) {
    const int64_t v = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x;
    if (v >= n_inst) return;
    long long acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0;
    const int k0 = node_ptr[v], k1 = node_ptr[v + 1];
    for (int k = k0; k < k1; ++k) {         // the instance's pins, stored contiguously
        const double* g = pin_g + static_cast<int64_t>(k) * C;
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] += llrint(g[c] * kFix);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) grad[v * C + c] = static_cast<float>(static_cast<double>(acc[c]) * kUnfix);
}

constexpr int kFinalBT = 1024;
constexpr int kFinalPer = (kMaxGrid + kFinalBT - 1) / kFinalBT;

__global__ void __launch_bounds__(kFinalBT) k_wa_final(const double* __restrict__ partial, int nparts, int npairs,
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

int wa_grid(int32_t n_nets) {
    int64_t g = (static_cast<int64_t>(n_nets) + kNetsPerWg - 1) / kNetsPerWg;
    return static_cast<int>(g < 1 ? 1 : (g > kMaxGrid ? kMaxGrid : g));
}

template <int P>
void wa_p(const WlIndex& w, const float* pos, double inv_g, double* wl, float* grad, hipStream_t s) {
    const ahr_netlist& nl = w.nl;
    constexpr int C = 2 * P;
    const int grid = wa_grid(nl.n_nets);
    const int32_t per = static_cast<int32_t>((static_cast<int64_t>(nl.n_nets) + grid - 1) / grid);
    DevBuf<double> partial, pin_g;
    partial.ensure(static_cast<size_t>(grid) * kMaxPairs, s);
    if (grad) pin_g.ensure(static_cast<size_t>(nl.n_pins > 0 ? nl.n_pins : 1) * C, s);
    const double bytes = static_cast<double>(nl.n_pins) * (4 + 8 + 4 * C + (grad ? 8 * C * 2 + 4 : 0)) +
                         static_cast<double>(nl.n_nets + 1) * 4 +
                         (grad ? static_cast<double>(nl.n_inst) * (4 + 4 * C) : 0.0);
    {
        ProfScope ps(kStageWa, s, bytes);
        hipLaunchKernelGGL(k_wa_nets<P>, dim3(grid), dim3(kBT), 0, s, pos, C, nl.net_ptr, nl.n_nets, per,
                           nl.pin_node, nl.pin_off, inv_g, partial.p, grad ? pin_g.p : nullptr, w.pin_slot.p);
        AHR_LAUNCHED("k_wa_nets");
        if (grad) {
            hipLaunchKernelGGL(k_wa_nodes<C>, dim3(grid_for(nl.n_inst, kBT)), dim3(kBT), 0, s, w.node_ptr.p,
                               pin_g.p, nl.n_inst, grad);
            AHR_LAUNCHED("k_wa_nodes");
        }
        hipLaunchKernelGGL(k_wa_final, dim3(1), dim3(kFinalBT), 0, s, partial.p, grid, P, wl);
        AHR_LAUNCHED("k_wa_final");
    }
    partial.release(s);
    pin_g.release(s);
}

}  // namespace

}  // namespace ahr

using ahr::fail;

extern "C" {

ahr_status ahr_wl_create(const ahr_netlist* nl, void* stream, ahr_wl** out) {
    if (!nl) return fail(AHR_EINVAL, "netlist is NULL");
    if (!out) return fail(AHR_EINVAL, "out is NULL");
    if (nl->n_inst <= 0 || nl->n_nets < 0 || nl->n_pins < 0 || nl->reserved0 != 0 || !nl->net_ptr ||
        (nl->n_pins > 0 && (!nl->pin_node || !nl->pin_off)))
        return fail(AHR_EINVAL, "bad netlist (counts, reserved0 or NULL arrays)");
    try {
        ahr::set_error(AHR_OK, "");
        hipStream_t s = static_cast<hipStream_t>(stream);
        auto* w = new ahr::WlIndex();
        w->nl = *nl;
        w->use_stream(s);
        try {
            AHR_HIP(hipGetDevice(&w->device));
            const int32_t n = nl->n_inst, P = nl->n_pins;
            ahr::DevBuf<int32_t> cnt;
            ahr::DevBuf<int32_t>& slot = w->pin_slot;
            ahr::DevBuf<int64_t> tmp;
            cnt.ensure(static_cast<size_t>(n) + 1, s);
            slot.ensure(static_cast<size_t>(P > 0 ? P : 1), s);
            tmp.ensure(ahr::scan_tmp_elems(n), s);
            w->node_ptr.ensure(static_cast<size_t>(n) + 1, s);
            w->node_pins.ensure(static_cast<size_t>(P > 0 ? P : 1), s);
            ahr::fill_i32(cnt.p, n, 0, s);
            if (P > 0) {
                hipLaunchKernelGGL(ahr::k_pin_slots, dim3(ahr::grid_for(P, ahr::kBT)), dim3(ahr::kBT), 0, s,
                                   nl->pin_node, P, cnt.p, slot.p);
                AHR_LAUNCHED("k_pin_slots");
            }
            ahr::scan_i32_to_i32(cnt.p, w->node_ptr.p, n, tmp.p, s);
            if (P > 0) {
                hipLaunchKernelGGL(ahr::k_pin_scatter, dim3(ahr::grid_for(P, ahr::kBT)), dim3(ahr::kBT), 0, s,
                                   nl->pin_node, P, slot.p, w->node_ptr.p, w->node_pins.p);
                AHR_LAUNCHED("k_pin_scatter");
            }
            cnt.release(s);
            tmp.release(s);
            AHR_HIP(hipStreamSynchronize(s));
        } catch (...) {
            delete w;
            throw;
        }
        *out = reinterpret_cast<ahr_wl*>(w);
        ahr::flush_frees();
        return AHR_OK;
    } catch (const ahr::Error& e) {
        ahr::flush_frees();
        return fail(e.code, e.msg);
    } catch (...) {
        ahr::flush_frees();
        return fail(AHR_EDEVICE, "unexpected exception");
    }
}

ahr_status ahr_wa(ahr_wl* h, const float* g, int32_t ncols, float gamma, double* wl, float* grad, void* stream) {
    if (!h) return fail(AHR_EINVAL, "wirelength index is NULL");
    if (!g || !wl) return fail(AHR_EINVAL, "g/wl is NULL");
    if (ncols != 2 && ncols != 4 && ncols != 8) return fail(AHR_EINVAL, "ncols must be 2, 4 or 8");
    if (!(gamma > 0.f) || !std::isfinite(gamma)) return fail(AHR_EINVAL, "gamma must be positive and finite");
    try {
        ahr::set_error(AHR_OK, "");
        const auto* w = reinterpret_cast<const ahr::WlIndex*>(h);
        hipStream_t s = static_cast<hipStream_t>(stream);
        w->use_stream(s);
        const double inv_g = 1.0 / static_cast<double>(gamma);
        switch (ncols) {
            case 2: ahr::wa_p<1>(*w, g, inv_g, wl, grad, s); break;
            case 4: ahr::wa_p<2>(*w, g, inv_g, wl, grad, s); break;
            default: ahr::wa_p<4>(*w, g, inv_g, wl, grad, s); break;
        }
        ahr::flush_frees();
        return AHR_OK;
    } catch (const ahr::Error& e) {
        ahr::flush_frees();
        return fail(e.code, e.msg);
    } catch (...) {
        ahr::flush_frees();
        return fail(AHR_EDEVICE, "unexpected exception");
    }
}

void ahr_wl_destroy(ahr_wl* h) {
    if (!h) return;
    try {
        delete reinterpret_cast<ahr::WlIndex*>(h);
    } catch (...) {
    }
    ahr::flush_frees();
}

}  // extern "C"
