// Weighted-average (WA) wirelength and its gradient (Section II-B of the
// paper, "Wirelength model"): for each net and axis the exponentially
// weighted means of the pin coordinates with weights exp(+x/gamma) (smooth
// maximum) and exp(-x/gamma) (smooth minimum); W sums their differences over
// nets and both axes.  This is the wirelength term of the electrostatic
// global placer that consumes the initializer's placement.
//
// Numbers: coordinates, sums and ratios in float64; each weight is taken
// relative to the net's extreme coordinate (exp((x - max)/gamma),
// exp((min - x)/gamma), which cancels in every ratio) and exponentiated in
// float32 (arguments <= 0, values in (0, 1], relative error ~1e-7): the
// weights are what the placer's gradient step needs, and float64
// exponentials cost the pass several times its memory time.  Gradient of pin i:
//   p+_i (1 + (x_i - xbar+)/gamma) - p-_i (1 - (x_i - xbar-)/gamma),
// p+-_i the pin's normalised weight.  An instance's gradient is the sum over
// its pins, added in int64 fixed point (2^-40 units), so the order in which
// the node pass meets the pins does not change the result.
//
// Layout: an index built once per netlist (ahr_wl_create) lists every
// instance's pins (node_ptr / node_pins), the nets of at most 64 pins in
// ascending degree (a stable bucket sort, so the lanes of a wave mostly
// meet nets of one degree and run the same trip counts) and the larger nets.
// One call is four kernels: the small-net pass (one thread per net: no lane
// idles on a short net and no cross-lane reduction; nets of at most 8 pins
// keep their pins in registers), the big-net pass (one workgroup per net),
// both writing net totals into workgroup partials and per-pin gradients into
// a [pins][ncols] float64 buffer in pin order; the node pass (one thread per
// instance gathers its pins' rows); and the fixed-order reduction of the
// partials.
#include <cmath>

#include "ahr_internal.hpp"
#include "device_util.hpp"

namespace ahr {

namespace {

constexpr int kBT = 256;
constexpr int kReg = 8;             // nets of up to kReg pins keep their pins in registers
constexpr int kMaxPairs = 4;
constexpr double kFix = 1099511627776.0;          // 2^40
constexpr double kUnfix = 1.0 / 1099511627776.0;

struct WlIndex {
    ahr_netlist nl;
    DevBuf<int32_t> node_ptr;     // [n_inst + 1]
    DevBuf<int32_t> node_pins;    // [n_pins] pins of each instance (order within an instance unspecified)
    DevBuf<int32_t> small;        // nets of 1..kWave pins, by ascending degree, ascending within a degree
    int32_t n_small = 0;
    DevBuf<int32_t> big;          // nets of more than kWave pins, ascending
    int32_t n_big = 0;
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
        small.release(s);
        big.release(s);
    }
};

// flag[e] = 1 for a net of more than kWave pins; key[e] = its degree for
// one of 1..kWave pins, -1 otherwise (the bucket sort's key).
__global__ void k_net_classes(const int32_t* __restrict__ net_ptr, int32_t n_nets, int32_t* __restrict__ flag,
                              int32_t* __restrict__ key) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e < n_nets) {
        const int32_t d = net_ptr[e + 1] - net_ptr[e];
        flag[e] = d > kWave ? 1 : 0;
        key[e] = d >= 1 && d <= kWave ? d : -1;
    }
}

__global__ void k_pin_slots(const int32_t* __restrict__ pin_node, int32_t n_pins, int32_t* __restrict__ cnt,
                            int32_t* __restrict__ slot) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p < n_pins) slot[p] = atomicAdd(&cnt[pin_node[p]], 1);
}

__global__ void k_pin_scatter(const int32_t* __restrict__ pin_node, int32_t n_pins,
                              const int32_t* __restrict__ slot, const int32_t* __restrict__ node_ptr,
                              int32_t* __restrict__ node_pins) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p < n_pins) node_pins[node_ptr[pin_node[p]] + slot[p]] = static_cast<int32_t>(p);
}

// exp(a) for a <= 0, in float32.
__device__ __forceinline__ double wexp(double a) { return static_cast<double>(expf(static_cast<float>(a))); }

// Coordinate of pin p in column c: instance position + pin offset (x or y).
__device__ __forceinline__ double pin_coord(const float* pos, int ncols, const int32_t* pin_node, const float* pin_off,
                                            int p, int c) {
    return static_cast<double>(pos[static_cast<int64_t>(pin_node[p]) * ncols + c]) +
           static_cast<double>(pin_off[2 * p + (c & 1)]);
}

// One net and one column at a time (only that column's sums are live, so the
// kernel keeps its registers few and its occupancy high).
struct ColAcc {
    double hi, lo;      // extremes
    double sp, tp;      // sum exp((x-hi)/g), sum x exp((x-hi)/g)
    double sm, tm;      // sum exp((lo-x)/g), sum x exp((lo-x)/g)
};

__device__ __forceinline__ double gpin(double x, const ColAcc& a, double inv_g) {
    const double xp = a.tp / a.sp, xm = a.tm / a.sm;
    const double pp = wexp((x - a.hi) * inv_g) / a.sp, pm = wexp((a.lo - x) * inv_g) / a.sm;
    return pp * (1.0 + (x - xp) * inv_g) - pm * (1.0 - (x - xm) * inv_g);
}

// One row of C float32 coordinates.
template <int C>
__device__ __forceinline__ void load_row(const float* p, float* v) {
    if constexpr (C == 2) {
        const float2 t = *reinterpret_cast<const float2*>(p);
        v[0] = t.x;
        v[1] = t.y;
    } else {
#pragma unroll
        for (int h = 0; h < C / 4; ++h) {
            const float4 t = reinterpret_cast<const float4*>(p)[h];
            v[4 * h] = t.x;
            v[4 * h + 1] = t.y;
            v[4 * h + 2] = t.z;
            v[4 * h + 3] = t.w;
        }
    }
}

// The D pins from p0 (indexes past the net's last pin p1 - 1 are clamped to
// it) of a net: node rows and offsets, every load issued before any is used.
template <int C, int D>
__device__ __forceinline__ void gather_pins(const float* __restrict__ pos, const int32_t* __restrict__ pin_node,
                                            const float* __restrict__ pin_off, int p0, int p1, float (&v)[D][C],
                                            float2 (&off)[D]) {
    int node[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const int p = p0 + k < p1 ? p0 + k : p1 - 1;
        node[k] = pin_node[p];
        off[k] = reinterpret_cast<const float2*>(pin_off)[p];
    }
#pragma unroll
    for (int k = 0; k < D; ++k) load_row<C>(pos + static_cast<int64_t>(node[k]) * C, v[k]);
}

__device__ __forceinline__ double coord(const float (&v), float2 off, int c) {
    return static_cast<double>(v) + static_cast<double>((c & 1) ? off.y : off.x);
}

// A net of d <= D pins (D the wave's bound), its pins in registers: per
// column pair the extremes (clamped repeats of the last pin change no
// extreme), the shifted sums over its d pins, the pair's WA term, and each
// pin's gradient from the weights already taken (1/sp and 1/sm once per net
// and column).
template <int P, int D>
__device__ __forceinline__ void wa_net_regs(const float* __restrict__ pos, const int32_t* __restrict__ pin_node,
                                            const float* __restrict__ pin_off, int p0, int d, double inv_g,
                                            double* tot, double* __restrict__ pin_g) {
    constexpr int C = 2 * P;
    float v[D][C];
    float2 off[D];
    gather_pins<C, D>(pos, pin_node, pin_off, p0, p0 + d, v, off);
#pragma unroll
    for (int q = 0; q < P; ++q) {
        double hi[2], lo[2], sp[2], tp[2], sm[2], tm[2];
        float ep[D][2], em[D][2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            hi[c] = -1e300;
            lo[c] = 1e300;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double x = coord(v[k][2 * q + c], off[k], c);
                hi[c] = x > hi[c] ? x : hi[c];
                lo[c] = x < lo[c] ? x : lo[c];
            }
            sp[c] = tp[c] = sm[c] = tm[c] = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double x = coord(v[k][2 * q + c], off[k], c);
                ep[k][c] = expf(static_cast<float>((x - hi[c]) * inv_g));
                em[k][c] = expf(static_cast<float>((lo[c] - x) * inv_g));
                if (k < d) {
                    sp[c] += ep[k][c];
                    tp[c] += x * ep[k][c];
                    sm[c] += em[k][c];
                    tm[c] += x * em[k][c];
                }
            }
        }
        tot[q] += (tp[0] / sp[0] - tm[0] / sm[0]) + (tp[1] / sp[1] - tm[1] / sm[1]);
        if (!pin_g) continue;
        double rsp[2], rsm[2], xp[2], xm[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            rsp[c] = 1.0 / sp[c];
            rsm[c] = 1.0 / sm[c];
            xp[c] = tp[c] * rsp[c];
            xm[c] = tm[c] * rsm[c];
        }
#pragma unroll
        for (int k = 0; k < D; ++k)
            if (k < d) {
                double g[2];
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const double x = coord(v[k][2 * q + c], off[k], c);
                    const double pp = static_cast<double>(ep[k][c]) * rsp[c], pm = static_cast<double>(em[k][c]) * rsm[c];
                    g[c] = pp * (1.0 + (x - xp[c]) * inv_g) - pm * (1.0 - (x - xm[c]) * inv_g);
                }
                *reinterpret_cast<double2*>(pin_g + static_cast<int64_t>(p0 + k) * C + 2 * q) = make_double2(g[0], g[1]);
            }
    }
}

// A net of more than kReg pins (up to a wave's worth): kReg pins at a time
// (loads clamped and all in flight), three passes per column pair --
// extremes, shifted sums, gradients.
template <int P>
__device__ __forceinline__ void wa_net_loop(const float* __restrict__ pos, const int32_t* __restrict__ pin_node,
                                            const float* __restrict__ pin_off, int p0, int d, double inv_g,
                                            double* tot, double* __restrict__ pin_g) {
    constexpr int C = 2 * P, D = kReg;
    const int p1 = p0 + d;
    double hi[C], lo[C], sp[C], tp[C], sm[C], tm[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        hi[c] = -1e300;
        lo[c] = 1e300;
        sp[c] = tp[c] = sm[c] = tm[c] = 0;
    }
    float v[D][C];
    float2 off[D];
    for (int b = p0; b < p1; b += D) {
        gather_pins<C, D>(pos, pin_node, pin_off, b, p1, v, off);
#pragma unroll
        for (int k = 0; k < D; ++k)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const double x = coord(v[k][c], off[k], c);
                hi[c] = x > hi[c] ? x : hi[c];
                lo[c] = x < lo[c] ? x : lo[c];
            }
    }
    for (int b = p0; b < p1; b += D) {
        gather_pins<C, D>(pos, pin_node, pin_off, b, p1, v, off);
#pragma unroll
        for (int k = 0; k < D; ++k)
            if (b + k < p1)
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const double x = coord(v[k][c], off[k], c);
                    const double ep = wexp((x - hi[c]) * inv_g), em = wexp((lo[c] - x) * inv_g);
                    sp[c] += ep;
                    tp[c] += x * ep;
                    sm[c] += em;
                    tm[c] += x * em;
                }
    }
#pragma unroll
    for (int q = 0; q < P; ++q)
        tot[q] += (tp[2 * q] / sp[2 * q] - tm[2 * q] / sm[2 * q]) + (tp[2 * q + 1] / sp[2 * q + 1] - tm[2 * q + 1] / sm[2 * q + 1]);
    if (!pin_g) return;
    ColAcc a[C];
#pragma unroll
    for (int c = 0; c < C; ++c) a[c] = ColAcc{hi[c], lo[c], sp[c], tp[c], sm[c], tm[c]};
    for (int b = p0; b < p1; b += D) {
        gather_pins<C, D>(pos, pin_node, pin_off, b, p1, v, off);
#pragma unroll
        for (int k = 0; k < D; ++k)
            if (b + k < p1)
#pragma unroll
                for (int q = 0; q < P; ++q)
                    *reinterpret_cast<double2*>(pin_g + static_cast<int64_t>(b + k) * C + 2 * q) =
                        make_double2(gpin(coord(v[k][2 * q], off[k], 0), a[2 * q], inv_g),
                                     gpin(coord(v[k][2 * q + 1], off[k], 1), a[2 * q + 1], inv_g));
    }
}

// One net per thread.  The list is sorted by degree, so the lanes of a wave
// hold nets of about one degree: the wave's largest degree picks how many
// pins each lane gathers at once (2, 3, 4 or kReg in registers; more than
// kReg in passes).  Workgroup totals to partial[blockIdx.x].
template <int P>
__global__ void __launch_bounds__(kBT) k_wa_small(const float* __restrict__ pos, int ncols,
                                                  const int32_t* __restrict__ net_ptr,
                                                  const int32_t* __restrict__ list, int32_t n_list,
                                                  const int32_t* __restrict__ pin_node,
                                                  const float* __restrict__ pin_off, double inv_g,
                                                  double* __restrict__ partial, double* __restrict__ pin_g) {
    __shared__ double red[kBT / kWave];
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x;
    double tot[P];
#pragma unroll
    for (int q = 0; q < P; ++q) tot[q] = 0;
    int p0 = 0, d = 0;
    if (i < n_list) {
        const int e = list[i];
        p0 = net_ptr[e];
        d = net_ptr[e + 1] - p0;
    }
    const int dmax = wave_max(d);
    if (d > 0) {
        if (dmax <= 2) wa_net_regs<P, 2>(pos, pin_node, pin_off, p0, d, inv_g, tot, pin_g);
        else if (dmax <= 3) wa_net_regs<P, 3>(pos, pin_node, pin_off, p0, d, inv_g, tot, pin_g);
        else if (dmax <= 4) wa_net_regs<P, 4>(pos, pin_node, pin_off, p0, d, inv_g, tot, pin_g);
        else if (dmax <= kReg) wa_net_regs<P, kReg>(pos, pin_node, pin_off, p0, d, inv_g, tot, pin_g);
        else wa_net_loop<P>(pos, pin_node, pin_off, p0, d, inv_g, tot, pin_g);
    }
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const double s2 = block_sum_f64<kBT>(tot[q], red);
        if (threadIdx.x == 0) partial[static_cast<int64_t>(blockIdx.x) * kMaxPairs + q] = s2;
    }
}

// Running (shifted) exponential sums: value m (the shift: the largest x so
// far for the maximum side, the smallest for the minimum side), sum of
// exp(+-(x - m)/g) and of x times it; merging rescales the side with the
// smaller (larger) shift.  One pass gives what the three-pass form gives.
struct Run {
    double m, s, t;
};

__device__ __forceinline__ void run_add(Run& r, double x, double sgn_inv_g) {
    // sgn_inv_g = +1/g (maximum side) or -1/g (minimum side)
    const double q = (x - r.m) * sgn_inv_g;
    if (q > 0) {            // new extreme: rescale what is there
        const double f = wexp(-q);
        r.s = r.s * f + 1.0;
        r.t = r.t * f + x;
        r.m = x;
    } else {
        const double e = wexp(q);
        r.s += e;
        r.t += x * e;
    }
}

__device__ __forceinline__ Run run_merge(Run a, Run b, double sgn_inv_g) {
    if (b.s == 0) return a;
    if (a.s == 0) return b;
    if ((b.m - a.m) * sgn_inv_g > 0) {
        Run t = a;
        a = b;
        b = t;
    }
    const double f = wexp((b.m - a.m) * sgn_inv_g);
    return Run{a.m, a.s + b.s * f, a.t + b.t * f};
}

// The nets above kWave pins, one workgroup each (listed once per index):
// one pass for the shifted sums of every column, one for the gradients.
template <int P>
__global__ void __launch_bounds__(kBT) k_wa_big(const float* __restrict__ pos, int ncols,
                                                const int32_t* __restrict__ net_ptr, const int32_t* __restrict__ big,
                                                const int32_t* __restrict__ pin_node,
                                                const float* __restrict__ pin_off, double inv_g,
                                                double* __restrict__ partial, double* __restrict__ pin_g) {
    __shared__ Run red[2 * P][2][kBT / kWave];
    const int e = big[blockIdx.x];
    const int p0 = net_ptr[e], p1 = net_ptr[e + 1];
    Run rp[2 * P], rm[2 * P];
#pragma unroll
    for (int c = 0; c < 2 * P; ++c) {
        rp[c] = Run{-1e300, 0, 0};
        rm[c] = Run{1e300, 0, 0};
    }
    for (int p = p0 + threadIdx.x; p < p1; p += kBT) {
#pragma unroll
        for (int c = 0; c < 2 * P; ++c) {
            const double x = pin_coord(pos, ncols, pin_node, pin_off, p, c);
            if (rp[c].s == 0) {
                rp[c] = Run{x, 1.0, x};
                rm[c] = Run{x, 1.0, x};
            } else {
                run_add(rp[c], x, inv_g);
                run_add(rm[c], x, -inv_g);
            }
        }
    }
    // wave then workgroup merges, in a fixed order
#pragma unroll
    for (int c = 0; c < 2 * P; ++c) {
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
            Run a{__shfl_xor(rp[c].m, o), __shfl_xor(rp[c].s, o), __shfl_xor(rp[c].t, o)};
            Run b{__shfl_xor(rm[c].m, o), __shfl_xor(rm[c].s, o), __shfl_xor(rm[c].t, o)};
            // lane pairs merge in lane order so both lanes hold the same bits
            rp[c] = (lane_id() & o) ? run_merge(a, rp[c], inv_g) : run_merge(rp[c], a, inv_g);
            rm[c] = (lane_id() & o) ? run_merge(b, rm[c], -inv_g) : run_merge(rm[c], b, -inv_g);
        }
        if (lane_id() == 0) {
            red[c][0][wave_id()] = rp[c];
            red[c][1][wave_id()] = rm[c];
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 2 * P; ++c) {
        rp[c] = red[c][0][0];
        rm[c] = red[c][1][0];
        for (int w = 1; w < kBT / kWave; ++w) {
            rp[c] = run_merge(rp[c], red[c][0][w], inv_g);
            rm[c] = run_merge(rm[c], red[c][1][w], -inv_g);
        }
    }
    if (pin_g) {
        for (int p = p0 + threadIdx.x; p < p1; p += kBT) {
            const int64_t k = static_cast<int64_t>(p) * ncols;
#pragma unroll
            for (int c = 0; c < 2 * P; ++c) {
                const double x = pin_coord(pos, ncols, pin_node, pin_off, p, c);
                const ColAcc a{rp[c].m, rm[c].m, rp[c].s, rp[c].t, rm[c].s, rm[c].t};
                pin_g[k + c] = gpin(x, a, inv_g);
            }
        }
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < P; ++c)
            partial[static_cast<int64_t>(blockIdx.x) * kMaxPairs + c] =
                (rp[2 * c].t / rp[2 * c].s - rm[2 * c].t / rm[2 * c].s) +
                (rp[2 * c + 1].t / rp[2 * c + 1].s - rm[2 * c + 1].t / rm[2 * c + 1].s);
    }
}

// Gradient of every instance: the exact (int64, 2^-40 units) sum of its
// pins' gradients, rounded once to float32.
template <int C>
__global__ void __launch_bounds__(kBT) k_wa_nodes(const int32_t* __restrict__ node_ptr,
                                                  const int32_t* __restrict__ node_pins,
                                                  const double* __restrict__ pin_g, int32_t n_inst,
                                                  float* __restrict__ grad) {
    const int64_t v = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x;
    if (v >= n_inst) return;
    long long acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0;
    const int k0 = node_ptr[v], k1 = node_ptr[v + 1];
    // kB pins at a time, every load in flight (indexes clamped to the last
    // pin; the repeats are not added)
    constexpr int kB = 4;
    for (int b = k0; b < k1; b += kB) {
        int pin[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) pin[u] = node_pins[b + u < k1 ? b + u : k1 - 1];
        double g[kB][C];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const double2* r = reinterpret_cast<const double2*>(pin_g + static_cast<int64_t>(pin[u]) * C);
#pragma unroll
            for (int h = 0; h < C / 2; ++h) {
                const double2 t = r[h];
                g[u][2 * h] = t.x;
                g[u][2 * h + 1] = t.y;
            }
        }
#pragma unroll
        for (int u = 0; u < kB; ++u)
            if (b + u < k1)
#pragma unroll
                for (int c = 0; c < C; ++c) acc[c] += llrint(g[u][c] * kFix);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) grad[v * C + c] = static_cast<float>(static_cast<double>(acc[c]) * kUnfix);
}

constexpr int kFinalBT = 1024;

// The partials in a fixed order: thread t adds partials t, t + kFinalBT, ...
// in turn, then a fixed block reduction.
__global__ void __launch_bounds__(kFinalBT) k_wa_final(const double* __restrict__ partial, int nparts, int npairs,
                                                       double* __restrict__ out) {
    __shared__ double red[kFinalBT / kWave];
    for (int c = 0; c < npairs; ++c) {
        double s = 0;
        for (int b = threadIdx.x; b < nparts; b += kFinalBT) s += partial[static_cast<int64_t>(b) * kMaxPairs + c];
        s = block_sum_f64<kFinalBT>(s, red);
        if (threadIdx.x == 0) out[c] = s;
    }
}

template <int P>
void wa_p(const WlIndex& w, const float* pos, double inv_g, double* wl, float* grad, hipStream_t s) {
    const ahr_netlist& nl = w.nl;
    constexpr int C = 2 * P;
    const int grid = static_cast<int>((static_cast<int64_t>(w.n_small) + kBT - 1) / kBT);
    DevBuf<double> partial, pin_g;
    partial.ensure(static_cast<size_t>(grid + w.n_big + 1) * kMaxPairs, s);
    if (grad) pin_g.ensure(static_cast<size_t>(nl.n_pins > 0 ? nl.n_pins : 1) * C, s);
    const double bytes = static_cast<double>(nl.n_pins) * (4 + 8 + 4 * C + (grad ? 8 * C * 2 + 4 : 0)) +
                         static_cast<double>(nl.n_nets + 1) * 4 +
                         (grad ? static_cast<double>(nl.n_inst) * (4 + 4 * C) : 0.0);
    {
        ProfScope ps(kStageWa, s, bytes);
        if (grid) {
            hipLaunchKernelGGL(k_wa_small<P>, dim3(grid), dim3(kBT), 0, s, pos, C, nl.net_ptr, w.small.p, w.n_small,
                               nl.pin_node, nl.pin_off, inv_g, partial.p, grad ? pin_g.p : nullptr);
            AHR_LAUNCHED("k_wa_small");
        }
        if (w.n_big) {
            hipLaunchKernelGGL(k_wa_big<P>, dim3(w.n_big), dim3(kBT), 0, s, pos, C, nl.net_ptr, w.big.p, nl.pin_node,
                               nl.pin_off, inv_g, partial.p + static_cast<int64_t>(grid) * kMaxPairs,
                               grad ? pin_g.p : nullptr);
            AHR_LAUNCHED("k_wa_big");
        }
        if (grad) {
            hipLaunchKernelGGL(k_wa_nodes<C>, dim3(grid_for(nl.n_inst, kBT)), dim3(kBT), 0, s, w.node_ptr.p,
                               w.node_pins.p, pin_g.p, nl.n_inst, grad);
            AHR_LAUNCHED("k_wa_nodes");
        }
        hipLaunchKernelGGL(k_wa_final, dim3(1), dim3(kFinalBT), 0, s, partial.p, grid + w.n_big, P, wl);
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
            ahr::DevBuf<int32_t> cnt, slot;
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
            slot.release(s);
            // nets above kWave pins, ascending (a flag scan); the others by degree
            if (nl->n_nets > 0) {
                ahr::DevBuf<int32_t> flag, rank, key, start, a, b;
                flag.ensure(static_cast<size_t>(nl->n_nets) + 1, s);
                rank.ensure(static_cast<size_t>(nl->n_nets) + 1, s);
                key.ensure(static_cast<size_t>(nl->n_nets) + 1, s);
                tmp.ensure(ahr::scan_tmp_elems(nl->n_nets), s);
                hipLaunchKernelGGL(ahr::k_net_classes, dim3(ahr::grid_for(nl->n_nets, ahr::kBT)), dim3(ahr::kBT), 0,
                                   s, nl->net_ptr, nl->n_nets, flag.p, key.p);
                AHR_LAUNCHED("k_net_classes");
                w->n_big = static_cast<int32_t>(ahr::scan_i32_checked(flag.p, rank.p, nl->n_nets, tmp.p, s));
                w->big.ensure(static_cast<size_t>(w->n_big) + 1, s);
                ahr::list_rows(flag.p, rank.p, nl->n_nets, w->big.p, s);
                flag.release(s);
                rank.release(s);
                w->n_small = ahr::bucket_sort(key.p, nl->n_nets, ahr::kWave + 1, w->small, start, a, b, tmp, s);
                key.release(s);
                start.release(s);
                a.release(s);
                b.release(s);
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
