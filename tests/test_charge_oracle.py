"""CPU pins of the macro charge-density oracle (Section VI): closed-form
masses over the whole footprint for each model, the flat limits, the
Gaussian's erf product against a two-dimensional quadrature of its density,
additivity over a bin partition, the schedules' defining values and the
symmetry of the densities."""
import math

import numpy as np
import pytest
from scipy import integrate, special

import netlists as H
from oracle import charge_oracle as Q

W, HH = 6.0, 4.0          # a footprint [-3, 3] x [-2, 2]


def full(model, param):
    return Q.pair_mass(model, param, -W / 2, W / 2, -HH / 2, HH / 2, W, HH)


@pytest.mark.parametrize("eta", [0.3, 1.0, 2.5, 6.0])
def test_gaussian_mass_is_the_footprint_area(eta):
    # the normalisation of eq. "Gaussion_eta": mass w h over the footprint, for every eta
    assert math.isclose(full(Q.GAUSSIAN, eta), W * HH, rel_tol=1e-13)


def test_gaussian_erf_product_equals_quadrature_of_the_density():
    eta = 1.7
    f = lambda y, x: Q.density(Q.GAUSSIAN, eta, x, y, W, HH)
    for (x0, x1, y0, y1) in [(-3, -1, -2, 0.5), (0.2, 2.9, -1.1, 1.3), (-0.5, 0.5, 1.0, 2.0)]:
        v, _ = integrate.dblquad(f, x0, x1, y0, y1, epsabs=1e-14, epsrel=1e-13)
        assert math.isclose(Q.pair_mass(Q.GAUSSIAN, eta, x0, x1, y0, y1, W, HH), v, rel_tol=1e-11)


@pytest.mark.parametrize("sigma", [0.05, 0.4, 1.0, 3.0])
def test_exponential_mass_closed_form(sigma):
    # int over [-L/2, L/2] of exp(-tan^2(pi x/L)/(2 s^2)) dx = L e^a erfc(sqrt a), a = 1/(2 s^2)
    a = 1 / (2 * sigma * sigma)
    one = special.erfcx(math.sqrt(a))
    assert math.isclose(full(Q.EXPONENTIAL, sigma), W * HH * one * one, rel_tol=1e-10)


@pytest.mark.parametrize("k", [0.0, 0.4, 1.0])
def test_linear_mass_small_k(k):
    # the cone never reaches zero inside: mass = w h (1 - k E[r]) with E[r] over the
    # square [-1/2, 1/2]^2 of sqrt 2 sqrt(u^2 + v^2) = sqrt 2 (sqrt 2 + ln(1 + sqrt 2)) / 6
    er = math.sqrt(2) * (math.sqrt(2) + math.log(1 + math.sqrt(2))) / 6
    assert math.isclose(full(Q.LINEAR, k), W * HH * (1 - k * er), rel_tol=1e-10)


@pytest.mark.parametrize("k", [1.5, 3.0, 10.0])
def test_linear_mass_cone_inside(k):
    # k >= sqrt 2: the cone's base circle lies inside; its volume is base x height / 3
    assert math.isclose(full(Q.LINEAR, k), W * HH * math.pi / (6 * k * k), rel_tol=1e-9)


def test_sigmoid_mass_large_k():
    # k large: the tail beyond the square is below e^-40; the radial integral is
    # 2 pi (2/k^2) pi^2/12 in (s, t) = sqrt 2 (u, v) units, and du dv = ds dt / 2
    k = 60.0
    assert math.isclose(full(Q.SIGMOID, k), W * HH * math.pi ** 3 / (6 * k * k), rel_tol=1e-9)


def test_flat_limits():
    for model, p in [(Q.GAUSSIAN, 1e-12), (Q.EXPONENTIAL, math.inf), (Q.LINEAR, 0.0), (Q.SIGMOID, 0.0)]:
        assert math.isclose(Q.pair_mass(model, p, -1, 2, -0.5, 1.5, W, HH), 3 * 2, rel_tol=1e-12)
    for model, p in [(Q.EXPONENTIAL, 0.0), (Q.LINEAR, math.inf), (Q.SIGMOID, math.inf)]:
        assert Q.pair_mass(model, p, -1, 2, -0.5, 1.5, W, HH) == 0.0


def test_schedules():
    cp = Q.ChargeParams(model=Q.GAUSSIAN, T=100)
    for t in (0, 10, 20):
        cp.t = t
        beta = cp.beta_min + (cp.beta_max - cp.beta_min) * t / 100
        assert math.isclose(Q.schedule(cp), math.sqrt(2 * math.log(2)) / beta, rel_tol=1e-14)
    for t in (80, 100):
        cp.t = t
        a = t / 100
        assert math.isclose(Q.schedule(cp), math.sqrt(-2 * ((1 - a) * math.log(cp.r0) + a * math.log(cp.r1))),
                            rel_tol=1e-14)
    cp.t = 50                        # halfway through the smoothstep: w = 1/2, geometric mean
    eta_a = math.sqrt(-2 * (0.5 * math.log(cp.r0) + 0.5 * math.log(cp.r1)))
    eta_b = math.sqrt(2 * math.log(2)) / (cp.beta_min + (cp.beta_max - cp.beta_min) * 0.5)
    assert math.isclose(Q.schedule(cp), math.sqrt(eta_a * eta_b), rel_tol=1e-14)
    e = Q.ChargeParams(model=Q.EXPONENTIAL, T=300, sigma_factor=0.01)
    e.t = 300 * (1 - math.exp(-1))   # ln(1 - t/T) = -1
    assert math.isclose(Q.schedule(e), 0.01 * 300, rel_tol=1e-12)
    k = Q.ChargeParams(model=Q.SIGMOID, T=200, t=100, k_factor=2.5)
    assert math.isclose(Q.schedule(k), 2.5, rel_tol=1e-14)


@pytest.mark.parametrize("model", [Q.GAUSSIAN, Q.EXPONENTIAL, Q.LINEAR, Q.SIGMOID])
def test_bins_partition_the_footprint(model):
    """A macro inside the die: its bin masses add up to its footprint mass;
    mirrored bins (macro centred on a bin corner) carry equal mass."""
    nl = H.make([[0, 1]], 2, flags=[H.MACRO, 0], sizes=[[6, 4], [1, 1]], pos=[[0.0, 0.0], [5, 5]],
                die=(-8, -8, 8, 8))
    cp = Q.ChargeParams(model=model, t=120, T=300, nbx=8, nby=8, sigma_factor=0.005, k_factor=1.0)
    m = Q.bin_mass(nl, nl["g0"], cp)
    param = Q.schedule(cp)
    assert math.isclose(m.sum(), full(model, param), rel_tol=1e-10)
    g = m.reshape(8, 8)
    assert np.allclose(g, g[::-1, :], rtol=1e-10, atol=1e-14) and np.allclose(g, g[:, ::-1], rtol=1e-10, atol=1e-14)
    assert np.count_nonzero(g) == 8           # [-3, 3] x [-2, 2] over 2 x 2 bins: 4 columns, 2 rows
