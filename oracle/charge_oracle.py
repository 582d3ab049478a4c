"""FP64 CPU oracle of the macro charge-density models and their per-bin
integrals (Section VI of arXiv 2511.10073, "Macro-Schedule Global
Placement").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP library.

Each macro m of width w and height h carries an iteration-dependent charge
density rho_t(dx, dy) in local coordinates (offsets from its centre), on its
footprint |dx| <= w/2, |dy| <= h/2; its contribution to bin b at iteration
t is the integral of rho_t over the part of the bin inside the footprint
(Section VI, the closing equation).  The four models:

  * Section VI-A, eq. "Gaussion_eta": an area-normalised, truncated 2-D
    Gaussian, rho = 2 eta^2 / (pi erf^2(eta/sqrt 2)) exp(-2 eta^2 (dx^2/w^2 +
    dy^2/h^2)); its mass over the footprint is w h.  eta(t) follows the
    blended schedule of eq. "eta_t" (Scheme A: log-linear edge decay ratio
    r; Scheme B: linear normalised FWHM beta; smoothstep mixing).
  * Section VI-B, eq. "exp_sigma": rho = exp(-(tan^2(pi dx/w) +
    tan^2(pi dy/h)) / (2 sigma^2)), with sigma(t) = -sigma_factor T ln(1 -
    t/T) (eq. "sigma_t").
  * eq. "linear_k": rho = 1 - k sqrt(2 (dx^2/w^2 + dy^2/h^2)).
  * eq. "sigmoid_k": rho = 2 / (1 + exp(k sqrt(2 (dx^2/w^2 + dy^2/h^2)))).
    Both with k(t) = k_factor / tan(pi t / (2T)).

Readings (the paper is silent or leaves these open):
  * the linear model is clipped below at zero, max(0, 1 - k r): a density is
    not negative, and the model restores charge from the centre outwards;
  * every model is restricted to the macro's footprint (stated for the
    Gaussian) and bins tile the die as in the area hints; footprint parts
    outside the die fall in no bin;
  * the schedules' end points are limits: sigma(0) = 0 and k(0) = infinity
    leave no mass, sigma(T) = infinity and k(T) = 0 give the flat footprint
    rho = 1;
  * the Gaussian schedule's constants (r0, r1, beta_min, beta_max, alpha0,
    alpha1) are not printed: the defaults below are builder choices;
  * every macro of the netlist (movable or fixed) is counted, at its
    position in the given placement.

The Gaussian's bin integral is the product of two one-dimensional erf
differences (the definition integrated exactly); the exponential model's is
the product of two adaptive one-dimensional quadratures; the linear and
sigmoid models' are adaptive two-dimensional quadratures of the definitions.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy import integrate, special

GAUSSIAN, EXPONENTIAL, LINEAR, SIGMOID = 0, 1, 2, 3


@dataclasses.dataclass
class ChargeParams:
    model: int = EXPONENTIAL         # the paper's default (Section VII-B: exponential-like restoration)
    t: int = 0
    T: int = 300                     # schedule_iteration
    nbx: int = 32
    nby: int = 32
    sigma_factor: float = 0.005
    k_factor: float = 1.0
    r0: float = 1e-3                 # Scheme A: centre-to-boundary amplitude at alpha = 0 and 1
    r1: float = 0.9
    beta_min: float = 0.1            # Scheme B: normalised FWHM at alpha = 0 and 1
    beta_max: float = 1.0
    alpha0: float = 0.2              # smoothstep window of the blend
    alpha1: float = 0.8


def schedule(cp: ChargeParams) -> float:
    """The model parameter at iteration t: eta (eq. "eta_t"), sigma (eq.
    "sigma_t") or k (the shared k(t)).  inf / 0 at the end points as read."""
    a = cp.t / cp.T
    if cp.model == GAUSSIAN:
        log_r = (1 - a) * math.log(cp.r0) + a * math.log(cp.r1)
        eta_a = math.sqrt(-2 * log_r)
        beta = cp.beta_min + (cp.beta_max - cp.beta_min) * a
        eta_b = math.sqrt(2 * math.log(2)) / beta
        if a <= cp.alpha0:
            wgt = 0.0
        elif a >= cp.alpha1:
            wgt = 1.0
        else:
            z = (a - cp.alpha0) / (cp.alpha1 - cp.alpha0)
            wgt = 3 * z * z - 2 * z ** 3
        return eta_b ** (1 - wgt) * eta_a ** wgt
    if cp.model == EXPONENTIAL:
        if cp.t >= cp.T:
            return math.inf
        return -cp.sigma_factor * cp.T * math.log(1 - a)
    if cp.t <= 0:
        return math.inf
    if cp.t >= cp.T:
        return 0.0
    return cp.k_factor / math.tan(math.pi / 2 * a)


def density(model, param, dx, dy, w, h):
    """rho_t at local offsets (dx, dy) inside the footprint."""
    if model == GAUSSIAN:
        eta = param
        c = 2 * eta * eta / (math.pi * special.erf(eta / math.sqrt(2)) ** 2)
        return c * math.exp(-2 * eta * eta * (dx * dx / (w * w) + dy * dy / (h * h)))
    if model == EXPONENTIAL:
        s = param
        q = math.tan(math.pi * dx / w) ** 2 + math.tan(math.pi * dy / h) ** 2
        return math.exp(-q / (2 * s * s))
    r = math.sqrt(2 * (dx * dx / (w * w) + dy * dy / (h * h)))
    if model == LINEAR:
        return max(0.0, 1 - param * r)
    return 2 / (1 + math.exp(param * r)) if param * r < 700 else 0.0


def _gauss_1d(eta, a, b, L):
    """Integral of exp(-2 eta^2 x^2 / L^2) over [a, b]."""
    s = math.sqrt(2) * eta / L
    return math.sqrt(math.pi) / (2 * s) * (special.erf(s * b) - special.erf(s * a))


def _exp_1d(sigma, a, b, L):
    """Integral of exp(-tan^2(pi x / L) / (2 sigma^2)) over [a, b] inside
    [-L/2, L/2] (adaptive quadrature; the peak at 0 is given as a break)."""
    f = lambda x: math.exp(-math.tan(math.pi * x / L) ** 2 / (2 * sigma * sigma)) if abs(x) < L / 2 else 0.0
    pts = [0.0] if a < 0 < b else None
    v, _ = integrate.quad(f, a, b, points=pts, epsabs=1e-14 * L, epsrel=1e-13, limit=400)
    return v


def pair_mass(model, param, x0, x1, y0, y1, w, h):
    """Integral of rho over the local rectangle [x0, x1] x [y0, y1] (inside
    the footprint)."""
    if x1 <= x0 or y1 <= y0:
        return 0.0
    if model == GAUSSIAN:
        eta = param
        if eta < 1e-8:
            return (x1 - x0) * (y1 - y0)
        c = 2 * eta * eta / (math.pi * special.erf(eta / math.sqrt(2)) ** 2)
        return c * _gauss_1d(eta, x0, x1, w) * _gauss_1d(eta, y0, y1, h)
    if model == EXPONENTIAL:
        if param == 0:
            return 0.0
        if math.isinf(param):
            return (x1 - x0) * (y1 - y0)
        return _exp_1d(param, x0, x1, w) * _exp_1d(param, y0, y1, h)
    if math.isinf(param):
        return 0.0
    if param == 0:
        return (x1 - x0) * (y1 - y0)
    return _radial_2d(model, param, x0, x1, y0, y1, w, h)


def _radial_2d(model, k, x0, x1, y0, y1, w, h):
    """Iterated adaptive quadrature of the radial models over a rectangle,
    with the integrands' kinks given as break points: the cone tip at the
    centre and, for the linear model, the circle r = 1/k where the clipped
    density reaches zero (in y for each x, and in x where the circle ends)."""
    tol = dict(epsabs=1e-15 * w * h, epsrel=1e-13, limit=200)

    def inside(lo, hi, pts):
        return sorted({p for p in pts if lo < p < hi}) or None

    def inner(x):
        br = [0.0]
        if model == LINEAR:
            q = 1 / (2 * k * k) - x * x / (w * w)
            if q > 0:
                br += [h * math.sqrt(q), -h * math.sqrt(q)]
        v, _ = integrate.quad(lambda y: density(model, k, x, y, w, h), y0, y1, points=inside(y0, y1, br), **tol)
        return v

    bx = [0.0] + ([w / (math.sqrt(2) * k), -w / (math.sqrt(2) * k)] if model == LINEAR else [])
    v, _ = integrate.quad(inner, x0, x1, points=inside(x0, x1, bx), **tol)
    return v


def macro_ids(nl):
    return np.flatnonzero((nl["node_flags"].astype(np.int64) & 2) != 0)


def bin_mass(nl, pos, cp: ChargeParams, macros=None):
    """Per bin b (row-major by (by, bx)), the sum over macros of the integral
    of rho_t over the part of bin b inside the macro's footprint; the bins
    tile the die.  `macros` restricts the sum (default: every macro)."""
    d = nl["die"].astype(np.float64)
    bw, bh = (d[2] - d[0]) / cp.nbx, (d[3] - d[1]) / cp.nby
    param = schedule(cp)
    out = np.zeros(cp.nbx * cp.nby)
    size = nl["node_size"].astype(np.float64)
    for m in (macro_ids(nl) if macros is None else macros):
        cx, cy = float(np.float32(pos[m, 0])), float(np.float32(pos[m, 1]))
        w, h = size[m]
        for by in range(cp.nby):
            ylo, yhi = d[1] + by * bh, d[1] + (by + 1) * bh
            y0, y1 = max(ylo, cy - h / 2) - cy, min(yhi, cy + h / 2) - cy
            if y1 <= y0:
                continue
            for bx in range(cp.nbx):
                xlo, xhi = d[0] + bx * bw, d[0] + (bx + 1) * bw
                x0, x1 = max(xlo, cx - w / 2) - cx, min(xhi, cx + w / 2) - cx
                if x1 <= x0:
                    continue
                out[by * cp.nbx + bx] += pair_mass(cp.model, param, x0, x1, y0, y1, w, h)
    return out
