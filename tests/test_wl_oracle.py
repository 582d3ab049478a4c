"""CPU pins of the WA wirelength oracle (Section II-B, "Wirelength model"):
a closed form on two pins, the gamma -> 0 limit (HPWL, itself pinned by
brute force), the bound WA <= HPWL, central finite differences of the
gradient, translation invariance and the zero gradient sum of every net."""
import math

import numpy as np
import pytest

import netlists as H
from oracle import ahr_oracle as O
from oracle import wl_oracle as W
from synth import netlist as N


def test_two_pin_net_closed_form():
    # pins at 0 and d on one axis: xbar+ - xbar- = d (sigmoid(d/g) - sigmoid(-d/g)) = d tanh(d / 2g)
    d, dy, g = 3.0, -1.25, 0.8
    nl = H.make([[0, 1]], 2, pos=[[0.0, 0.0], [d, dy]])
    tot, per, grad = W.wa_wirelength(nl, nl["g0"], g)
    want = d * math.tanh(d / (2 * g)) + abs(dy) * math.tanh(abs(dy) / (2 * g))
    assert math.isclose(tot[0], want, rel_tol=1e-14)
    # d/dd [d tanh(d/2g)] = tanh(d/2g) + d/(2g) sech^2(d/2g): + on the far pin, - on the near one
    dd = math.tanh(d / (2 * g)) + d / (2 * g) / math.cosh(d / (2 * g)) ** 2
    ddy = math.tanh(abs(dy) / (2 * g)) + abs(dy) / (2 * g) / math.cosh(dy / (2 * g)) ** 2
    assert np.allclose(grad, [[-dd, ddy], [dd, -ddy]], rtol=1e-13, atol=0)


def test_single_pin_and_empty_nets_are_zero():
    nl = H.make([[0], [], [1, 2]], 3, pos=[[1.0, 2.0], [0.0, 0.0], [0.0, 1.0]])
    tot, per, grad = W.wa_wirelength(nl, nl["g0"], 0.5)
    assert per[0, 0] == 0.0 and per[1, 0] == 0.0
    assert np.all(grad[0] == 0)
    assert math.isclose(tot[0], math.tanh(1.0), rel_tol=1e-14)      # y gap 1, gamma 0.5


def test_small_gamma_reaches_hpwl():
    # integer pin sites, at least one apart: every non-extreme weight is e^-100 or smaller
    rng = np.random.default_rng(1)
    nl = N.generate(N.small(400, 12, ncols=4))
    G = np.round(nl["g0"] * 8).astype(np.float32)
    nl["pin_off"] = np.round(nl["pin_off"]).astype(np.float32)
    tot, per, _ = W.wa_wirelength(nl, G, 0.01, with_grad=False)
    hp, hper = O.hpwl(nl, G)
    # nets whose extreme coordinates are shared by two pins are still exact (equal values)
    assert np.allclose(per, hper, rtol=0, atol=1e-9)
    assert np.allclose(tot, hp, rtol=1e-12)


def test_wa_never_exceeds_hpwl():
    nl = N.generate(N.small(600, 13, ncols=4))
    for g in (0.1, 1.0, 10.0):
        _, per, _ = W.wa_wirelength(nl, nl["g0"], g, with_grad=False)
        _, hper = O.hpwl(nl, nl["g0"])
        assert np.all(per <= hper + 1e-9)
        assert np.all(per >= -1e-12)


def test_gradient_central_differences():
    nl = N.generate(N.small(60, 14, ncols=2))
    G = nl["g0"].astype(np.float64)
    g = 1.5
    _, _, grad = W.wa_wirelength(nl, G, g)
    rng = np.random.default_rng(0)
    eps = 1e-6
    for _ in range(40):
        i, c = int(rng.integers(nl["n_inst"])), int(rng.integers(2))
        Gp, Gm = G.copy(), G.copy()
        Gp[i, c] += eps
        Gm[i, c] -= eps
        fd = (W.wa_wirelength(nl, Gp, g, False)[0][0] - W.wa_wirelength(nl, Gm, g, False)[0][0]) / (2 * eps)
        assert abs(fd - grad[i, c]) <= 1e-6 * max(1.0, abs(grad[i, c])), (i, c, fd, grad[i, c])


def test_translation_invariance_and_zero_gradient_sum():
    nl = N.generate(N.small(300, 15, ncols=2))
    G = nl["g0"].astype(np.float64)
    t0, _, g0 = W.wa_wirelength(nl, G, 2.0)
    t1, _, g1 = W.wa_wirelength(nl, G + np.array([7.5, -3.25]), 2.0)
    assert np.allclose(t0, t1, rtol=1e-12)
    assert np.allclose(g0, g1, rtol=0, atol=1e-11)
    # each net's pin gradients sum to zero, so the instance gradients do too
    assert np.allclose(g0.sum(axis=0), 0.0, atol=1e-9)


@pytest.mark.parametrize("g", [0.05, 3.0])
def test_per_net_loop_brute_force(g):
    """A pure-Python loop over nets and pins straight from the definition
    (no shift by the maximum: small coordinates keep exp in range)."""
    nl = N.generate(N.small(120, 16, ncols=2))
    G = (nl["g0"].astype(np.float64) - nl["g0"].mean(axis=0)) * 0.01   # keep |x|/g small enough for plain exp
    tot, per, grad = W.wa_wirelength(nl, G, g)
    ptr, node, off = nl["net_ptr"], nl["pin_node"], nl["pin_off"].astype(np.float64)
    s = 0.0
    for e in range(len(ptr) - 1):
        for c in range(2):
            xs = [G[node[k], c] + off[k, c] for k in range(ptr[e], ptr[e + 1])]
            if not xs:
                continue
            wp = [math.exp(x / g) for x in xs]
            wm = [math.exp(-x / g) for x in xs]
            s += sum(x * w for x, w in zip(xs, wp)) / sum(wp) - sum(x * w for x, w in zip(xs, wm)) / sum(wm)
    assert math.isclose(tot[0], s, rel_tol=1e-11)
