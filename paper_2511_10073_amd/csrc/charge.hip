// Macro charge-density models and their per-bin integrals (Section VI of the
// paper, "Macro-Schedule Global Placement"): each macro's footprint carries
// an iteration-dependent density rho_t(dx, dy) (local offsets from its
// centre), and its contribution to bin b is the integral of rho_t over the
// part of b inside the footprint.  Models:
//   Gaussian (eq. "Gaussion_eta"): 2 eta^2/(pi erf^2(eta/sqrt 2)) exp(-2 eta^2
//     (dx^2/w^2 + dy^2/h^2)), eta(t) from the blended schedule (eq. "eta_t");
//   exponential (eq. "exp_sigma"): exp(-(tan^2(pi dx/w) + tan^2(pi dy/h)) /
//     (2 sigma^2)), sigma(t) = -sigma_factor T ln(1 - t/T) (eq. "sigma_t");
//   linear (eq. "linear_k"): max(0, 1 - k r); sigmoid (eq. "sigmoid_k"):
//     2/(1 + exp(k r)); r = sqrt(2 (dx^2/w^2 + dy^2/h^2)), k(t) = k_factor /
//     tan(pi t / 2T).  (The clip at zero of the linear model is a reading.)
//
// Bin integrals, in float64:
//   * Gaussian: the product of two erf differences (exact);
//   * exponential: separable; each factor is (w/pi) int e^{-a u^2}/(1+u^2) du
//     over u = tan(pi x/w), a = 1/(2 sigma^2), by Gauss-Legendre rules on
//     panels that follow the integrand's scales (the Gaussian width 1/sqrt a
//     and the Lorentzian width 1);
//   * linear and sigmoid: radial in s = sqrt 2 dx/w, t = sqrt 2 dy/h, so a
//     rectangle is a signed sum of four corner rectangles [0, s] x [0, t],
//     each two triangles with a vertex at the centre, integrated in polar
//     form: int F(R(theta)) dtheta with F(R) = int_0^R f(r) r dr.  For the
//     linear model F and the theta integral have closed forms (split where
//     the cone reaches zero); for the sigmoid, Gauss-Legendre in r and, in
//     u = tan theta, on panels [0, 1], [1, 2], [2, 4], ...
// One thread per (macro, bin) pair; the masses are added per bin in int64
// fixed point (2^-28 area units), so the sums do not depend on their order.
#include <cmath>

#include "ahr_internal.hpp"
#include "device_util.hpp"

namespace ahr {

namespace {

constexpr int kBT = 256;
constexpr double kFix = 268435456.0;   // 2^28
constexpr double kPi = 3.14159265358979323846;

// Gauss-Legendre rules of 16 and 32 points on [-1, 1], and the series of
// the sigmoid model's radial integral (below), computed on the host.
constexpr int kSigSeries = 20;
struct GLRules {
    double x16[16], w16[16], x32[32], w32[32];
    double sig[kSigSeries];   // G(U) = U^2/4 + sum_m sig[m-1] U^(2m+1), U <= 1
};

// Coefficients of U^(2m+1) in G(U) = int_0^U u / (1 + e^u) du.  Since
// u / (1 + e^u) = u/2 - (u/2) tanh(u/2) and tanh x = sum_n t_n x^n (odd n),
// G(U) = U^2/4 - sum_m t_(2m-1) U^(2m+1) / (4^m (2m+1)); the t_n follow
// from tanh' = 1 - tanh^2: t_1 = 1, n t_n = -sum_(i+j=n-1) t_i t_j.
void sigmoid_series(double* out) {
    double t[2 * kSigSeries + 2] = {0};
    t[1] = 1.0;
    for (int m = 1; m < kSigSeries; ++m) {
        const int n = 2 * m + 1;
        double acc = 0;
        for (int i = 1; i < n - 1; i += 2) acc += t[i] * t[n - 1 - i];
        t[n] = -acc / n;
    }
    double p4 = 1.0;
    for (int m = 1; m <= kSigSeries; ++m) {
        p4 *= 4.0;
        out[m - 1] = -t[2 * m - 1] / (p4 * (2 * m + 1));
    }
}

void legendre_rule(int n, double* x, double* w) {
    // Newton iteration on P_n from the Chebyshev-like first guesses
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2 / ((1 - z * z) * dp * dp);
    }
}

const GLRules& gl_rules() {
    static const GLRules r = [] {
        GLRules g{};
        legendre_rule(16, g.x16, g.w16);
        legendre_rule(32, g.x32, g.w32);
        sigmoid_series(g.sig);
        return g;
    }();
    return r;
}

struct ChargeArgs {
    GLRules gl;
    int model;
    double param;                 // eta, sigma or k at iteration t (inf allowed)
    double xl, yl, bw, bh;
    int32_t nbx, nby;
};

// ---------------------------------------------------------------- Gaussian

__device__ double gauss_pair(double eta, double x0, double x1, double y0, double y1, double w, double h) {
    if (eta < 1e-8) return (x1 - x0) * (y1 - y0);
    const double e = erf(eta * 0.70710678118654752440);
    const double c = 2 * eta * eta / (kPi * e * e);
    const double sx = 1.41421356237309504880 * eta / w, sy = 1.41421356237309504880 * eta / h;
    const double half_sqrt_pi = 0.88622692545275801365;
    const double ix = half_sqrt_pi / sx * (erf(sx * x1) - erf(sx * x0));
    const double iy = half_sqrt_pi / sy * (erf(sy * y1) - erf(sy * y0));
    return c * ix * iy;
}

// ---------------------------------------------------------------- exponential

template <class F>
__device__ double gl16(const GLRules& g, F f, double a, double b) {
    if (!(b > a)) return 0.0;
    const double m = 0.5 * (a + b), hh = 0.5 * (b - a);
    double s = 0;
    for (int i = 0; i < 16; ++i) s += g.w16[i] * f(m + hh * g.x16[i]);
    return hh * s;
}

template <class F>
__device__ double gl32(const GLRules& g, F f, double a, double b) {
    if (!(b > a)) return 0.0;
    const double m = 0.5 * (a + b), hh = 0.5 * (b - a);
    double s = 0;
    for (int i = 0; i < 32; ++i) s += g.w32[i] * f(m + hh * g.x32[i]);
    return hh * s;
}

// J(a, U) = int_0^U exp(-a u^2) / (1 + u^2) du, U may be infinite.
__device__ double exp_J(const GLRules& g, double a, double U) {
    if (a >= 1) {   // y = sqrt(a) u: exp(-y^2) / (1 + y^2 / a), cut where exp(-y^2) < 1e-21
        const double ra = sqrt(a);
        const double Y = U * ra < 7.0 ? U * ra : 7.0;
        return gl32(g, [a](double y) { return exp(-y * y) / (1 + y * y / a); }, 0.0, Y) / ra;
    }
    // J = atan(U) - K with K = int_0^U (1 - exp(-a u^2)) / (1 + u^2) du: panels
    // [0, 1], [1, 2], [2, 4], ... up to 1/sqrt(a), then t = 1/(sqrt(a) u)
    const double ra = sqrt(a), top = U < 1 / ra ? U : 1 / ra;
    double k = 0, lo = 0, hi = 1;
    while (lo < top) {
        const double b = hi < top ? hi : top;
        k += gl16(g, [a](double u) { return -expm1(-a * u * u) / (1 + u * u); }, lo, b);
        lo = b;
        hi *= 2;
    }
    if (U * ra > 1) {
        const double t0 = isinf(U) ? 0.0 : 1 / (ra * U);
        k += gl32(g, [a, ra](double t) { return (t > 0 ? -expm1(-1 / (t * t)) : 1.0) * ra / (a * t * t + 1); }, t0,
                  1.0);
    }
    return (isinf(U) ? kPi / 2 : atan(U)) - k;
}

// int_{x0}^{x1} exp(-tan^2(pi x / L) / (2 sigma^2)) dx, [x0, x1] inside [-L/2, L/2].
__device__ double exp_1d(const GLRules& g, double sigma, double x0, double x1, double L) {
    const double a = 1 / (2 * sigma * sigma);
    auto S = [&](double x) {
        if (x >= L / 2) return exp_J(g, a, INFINITY);
        if (x <= -L / 2) return -exp_J(g, a, INFINITY);
        const double u = tan(kPi * x / L);
        return copysign(exp_J(g, a, fabs(u)), u);
    };
    return L / kPi * (S(x1) - S(x0));
}

// ---------------------------------------------------------------- radial models

// Triangle 0 <= theta <= atan(t/s) under the edge x = s (s, t > 0) of
// max(0, 1 - k r): F(R) = R^2/2 - k R^3/3 up to R = 1/k, 1/(6k^2) beyond.
__device__ double linear_tri(double k, double s, double t) {
    if (!(s > 0) || !(t > 0)) return 0.0;
    const double fmax = 1 / (6 * k * k);
    if (k * s >= 1) return atan2(t, s) * fmax;
    auto closed = [&](double tn, double sc) {
        return s * s / 2 * tn - k * s * s * s / 6 * (sc * tn + log(sc + tn));
    };
    const double R = hypot(s, t);
    if (k * R <= 1) return closed(t / s, R / s);
    const double sc = 1 / (k * s), tn = sqrt(fmax_d(sc * sc - 1, 0.0));
    return closed(tn, sc) + (atan2(t, s) - atan(tn)) * fmax;
}

// F(R) = int_0^R 2 r / (1 + e^(k r)) dr = (2 / k^2) G(k R) in closed form:
// for U <= 1 the series of G (its terms fall like (U / pi)^(2m)), above
// G(U) = pi^2/12 - U ln(1 + e^-U) + Li2(-e^-U), the dilogarithm by its power
// series in x = -e^-U (|x| <= 1/e: 40 terms reach 1e-19).  Both agree with
// an adaptive quadrature of G to a few 1e-16.
__device__ double sigmoid_G(const GLRules& g, double U) {
    if (U <= 1.0) {
        const double u2 = U * U;
        double acc = 0;
        for (int m = kSigSeries - 1; m >= 0; --m) acc = acc * u2 + g.sig[m];
        return u2 / 4 + acc * u2 * U;
    }
    const double x = -exp(-U);
    double li = 0, xn = 1;
    for (int n = 1; n <= 40; ++n) {
        xn *= x;
        li += xn / static_cast<double>(n * n);
    }
    return 0.82246703342411321824 - U * log1p(-x) + li;    // pi^2 / 12
}

__device__ double sigmoid_F(const GLRules& g, double k, double R) {
    return 2.0 / (k * k) * sigmoid_G(g, k * R);
}

__device__ double sigmoid_tri(const GLRules& g, double k, double s, double t) {
    if (!(s > 0) || !(t > 0)) return 0.0;
    const double U = t / s;
    double tot = 0, lo = 0, hi = 1;
    while (lo < U) {
        const double b = hi < U ? hi : U;
        tot += gl16(g, [&](double u) { return sigmoid_F(g, k, s * sqrt(1 + u * u)) / (1 + u * u); }, lo, b);
        lo = b;
        hi *= 2;
    }
    return tot;
}

__device__ double radial_pair(const GLRules& g, int model, double k, double x0, double x1, double y0, double y1,
                              double w, double h) {
    auto tri = [&](double s, double t) {
        return model == AHR_CHARGE_LINEAR ? linear_tri(k, s, t) : sigmoid_tri(g, k, s, t);
    };
    auto corner = [&](double s, double t) {   // signed integral over [0, s] x [0, t]
        const double sg = copysign(1.0, s) * copysign(1.0, t);
        s = fabs(s);
        t = fabs(t);
        return sg * (tri(s, t) + tri(t, s));
    };
    const double c = 1.41421356237309504880;
    const double s0 = c * x0 / w, s1 = c * x1 / w, t0 = c * y0 / h, t1 = c * y1 / h;
    return w * h / 2 * (corner(s1, t1) - corner(s0, t1) - corner(s1, t0) + corner(s0, t0));
}

__device__ double pair_mass(const ChargeArgs& a, double x0, double x1, double y0, double y1, double w, double h) {
    const double p = a.param;
    switch (a.model) {
        case AHR_CHARGE_GAUSSIAN: return gauss_pair(p, x0, x1, y0, y1, w, h);
        case AHR_CHARGE_EXP:
            if (p == 0) return 0.0;
            if (isinf(p)) return (x1 - x0) * (y1 - y0);
            return exp_1d(a.gl, p, x0, x1, w) * exp_1d(a.gl, p, y0, y1, h);
        default:
            if (isinf(p)) return 0.0;
            if (p == 0) return (x1 - x0) * (y1 - y0);
            return radial_pair(a.gl, a.model, p, x0, x1, y0, y1, w, h);
    }
}

// ---------------------------------------------------------------- kernels

struct Span {
    int bx0, nx, by0, ny;
};

__device__ Span macro_span(const ChargeArgs& a, double cx, double cy, double w, double h) {
    // bins whose rectangle can meet the footprint, one more on each side
    // (pairs with an empty intersection contribute nothing)
    Span sp{0, 0, 0, 0};
    int bx0 = static_cast<int>(floor((cx - w / 2 - a.xl) / a.bw)) - 1;
    int bx1 = static_cast<int>(floor((cx + w / 2 - a.xl) / a.bw)) + 1;
    int by0 = static_cast<int>(floor((cy - h / 2 - a.yl) / a.bh)) - 1;
    int by1 = static_cast<int>(floor((cy + h / 2 - a.yl) / a.bh)) + 1;
    bx0 = bx0 < 0 ? 0 : bx0;
    by0 = by0 < 0 ? 0 : by0;
    bx1 = bx1 > a.nbx - 1 ? a.nbx - 1 : bx1;
    by1 = by1 > a.nby - 1 ? a.nby - 1 : by1;
    if (bx1 < bx0 || by1 < by0) return sp;
    sp.bx0 = bx0;
    sp.nx = bx1 - bx0 + 1;
    sp.by0 = by0;
    sp.ny = by1 - by0 + 1;
    return sp;
}

__device__ bool macro_geom(const float* pos, int ncols, const uint8_t* flags, const float* size, int64_t i,
                           double& cx, double& cy, double& w, double& h) {
    if (!(flags[i] & AHR_NODE_MACRO)) return false;
    cx = pos[i * ncols];
    cy = pos[i * ncols + 1];
    w = size[2 * i];
    h = size[2 * i + 1];
    return w > 0 && h > 0;
}

__global__ void __launch_bounds__(kBT) k_charge_count(ChargeArgs a, const float* __restrict__ pos, int ncols,
                                                      const uint8_t* __restrict__ flags,
                                                      const float* __restrict__ size, int32_t n,
                                                      int32_t* __restrict__ cnt) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x;
    if (i >= n) return;
    double cx, cy, w, h;
    int c = 0;
    if (macro_geom(pos, ncols, flags, size, i, cx, cy, w, h)) {
        const Span sp = macro_span(a, cx, cy, w, h);
        c = sp.nx * sp.ny;
    }
    cnt[i] = c;
}

__global__ void __launch_bounds__(kBT) k_charge_pairs(ChargeArgs a, const float* __restrict__ pos, int ncols,
                                                      const uint8_t* __restrict__ flags,
                                                      const float* __restrict__ size, int32_t n,
                                                      const int64_t* __restrict__ off, int64_t n_pairs,
                                                      unsigned long long* __restrict__ bin_q) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBT;
    for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x; p < n_pairs; p += stride) {
        int32_t lo = 0, hi = n;          // off[lo] <= p < off[hi]
        while (hi - lo > 1) {
            const int32_t mid = lo + (hi - lo) / 2;
            if (off[mid] <= p) lo = mid; else hi = mid;
        }
        double cx, cy, w, h;
        if (!macro_geom(pos, ncols, flags, size, lo, cx, cy, w, h)) continue;
        const Span sp = macro_span(a, cx, cy, w, h);
        const int j = static_cast<int>(p - off[lo]);
        const int bx = sp.bx0 + j % sp.nx, by = sp.by0 + j / sp.nx;
        const double xlo = a.xl + bx * a.bw, xhi = a.xl + (bx + 1) * a.bw;
        const double ylo = a.yl + by * a.bh, yhi = a.yl + (by + 1) * a.bh;
        const double x0 = fmax_d(xlo, cx - w / 2) - cx, x1 = fmin_d(xhi, cx + w / 2) - cx;
        const double y0 = fmax_d(ylo, cy - h / 2) - cy, y1 = fmin_d(yhi, cy + h / 2) - cy;
        if (!(x1 > x0) || !(y1 > y0)) continue;
        const double m = pair_mass(a, x0, x1, y0, y1, w, h);
        atomicAdd(&bin_q[static_cast<int64_t>(by) * a.nbx + bx], static_cast<unsigned long long>(llrint(m * kFix)));
    }
}

__global__ void k_fill_u64z(unsigned long long* __restrict__ p, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void k_charge_out(const unsigned long long* __restrict__ q, int64_t n, double* __restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x;
    if (i < n) out[i] = static_cast<double>(static_cast<long long>(q[i])) / kFix;
}

}  // namespace

double charge_schedule(const ahr_charge_params& cp) {
    const double a = static_cast<double>(cp.t) / cp.T;
    if (cp.model == AHR_CHARGE_GAUSSIAN) {
        const double log_r = (1 - a) * std::log(static_cast<double>(cp.r0)) + a * std::log(static_cast<double>(cp.r1));
        const double eta_a = std::sqrt(-2 * log_r);
        const double beta = cp.beta_min + (static_cast<double>(cp.beta_max) - cp.beta_min) * a;
        const double eta_b = std::sqrt(2 * std::log(2.0)) / beta;
        double wgt;
        if (a <= cp.alpha0) {
            wgt = 0.0;
        } else if (a >= cp.alpha1) {
            wgt = 1.0;
        } else {
            const double z = (a - cp.alpha0) / (static_cast<double>(cp.alpha1) - cp.alpha0);
            wgt = 3 * z * z - 2 * z * z * z;
        }
        return std::pow(eta_b, 1 - wgt) * std::pow(eta_a, wgt);
    }
    if (cp.model == AHR_CHARGE_EXP) {
        if (cp.t >= cp.T) return INFINITY;
        return -static_cast<double>(cp.sigma_factor) * cp.T * std::log(1 - a);
    }
    if (cp.t <= 0) return INFINITY;
    if (cp.t >= cp.T) return 0.0;
    return static_cast<double>(cp.k_factor) / std::tan(kPi / 2 * a);
}

void run_macro_charge(const ahr_netlist& nl, const float* pos, int32_t ncols, const ahr_charge_params& cp,
                      double* out, hipStream_t s) {
    ChargeArgs a;
    a.gl = gl_rules();
    a.model = cp.model;
    a.param = charge_schedule(cp);
    a.xl = nl.die[0];
    a.yl = nl.die[1];
    a.bw = (static_cast<double>(nl.die[2]) - static_cast<double>(nl.die[0])) / cp.nbx;
    a.bh = (static_cast<double>(nl.die[3]) - static_cast<double>(nl.die[1])) / cp.nby;
    a.nbx = cp.nbx;
    a.nby = cp.nby;
    const int32_t n = nl.n_inst;
    const int64_t nbins = static_cast<int64_t>(cp.nbx) * cp.nby;
    DevBuf<int32_t> cnt;
    DevBuf<int64_t> off, tmp;
    DevBuf<unsigned long long> q;
    cnt.ensure(static_cast<size_t>(n) + 1, s);
    off.ensure(static_cast<size_t>(n) + 1, s);
    tmp.ensure(scan_tmp_elems(n), s);
    q.ensure(static_cast<size_t>(nbins), s);
    hipLaunchKernelGGL(k_fill_u64z, dim3(grid_for(nbins, kBT)), dim3(kBT), 0, s, q.p, nbins);
    AHR_LAUNCHED("k_fill_u64z");
    hipLaunchKernelGGL(k_charge_count, dim3(grid_for(n, kBT)), dim3(kBT), 0, s, a, pos, ncols, nl.node_flags,
                       nl.node_size, n, cnt.p);
    AHR_LAUNCHED("k_charge_count");
    scan_i32_to_i64(cnt.p, off.p, n, tmp.p, s);
    const int64_t n_pairs = read_i64(off.p + n, s);
    if (n_pairs > 0) {
        const int64_t blocks = (n_pairs + kBT - 1) / kBT;
        hipLaunchKernelGGL(k_charge_pairs, dim3(static_cast<unsigned>(blocks < 65536 ? blocks : 65536)), dim3(kBT), 0,
                           s, a, pos, ncols, nl.node_flags, nl.node_size, n, off.p, n_pairs, q.p);
        AHR_LAUNCHED("k_charge_pairs");
    }
    hipLaunchKernelGGL(k_charge_out, dim3(grid_for(nbins, kBT)), dim3(kBT), 0, s, q.p, nbins, out);
    AHR_LAUNCHED("k_charge_out");
    cnt.release(s);
    off.release(s);
    tmp.release(s);
    q.release(s);
}

}  // namespace ahr
