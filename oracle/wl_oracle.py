"""FP64 CPU oracle of the weighted-average (WA) wirelength and its gradient.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP library.

Section II-B of arXiv 2511.10073, "Wirelength model": for a net e with pin
coordinates x_i, the smooth maximum and minimum are the exponentially
weighted means
    xbar+_e = sum_i x_i exp(x_i / gamma) / sum_i exp(x_i / gamma),
    xbar-_e = sum_i x_i exp(-x_i / gamma) / sum_i exp(-x_i / gamma),
likewise in y, and W = sum_e (xbar+_e - xbar-_e) + (ybar+_e - ybar-_e) with
smoothing parameter gamma.  Its gradient moves the instances of a net
towards each other.

Readings (the paper is silent on them):
  * pin coordinates are the instance position plus the pin offset, on the
    netlist's own pins (as for HPWL); net weights are not applied (the
    paper's W has none);
  * exp(x_i / gamma) is evaluated as exp((x_i - max_j x_j) / gamma) (and
    exp((min_j x_j - x_i) / gamma) for the minus side): the common factor
    cancels in each ratio, so the values are those of the definition, without
    overflow;
  * the gradient with respect to an instance is the sum over its pins;
  * columns 2c, 2c+1 are the x and y of placement c, as everywhere else.
"""
from __future__ import annotations

import numpy as np


def _net_means(px, starts, net_of_pin, gamma, sign):
    """Exponentially weighted mean of each net's coordinates with weights
    exp(sign * x / gamma) (sign = +1: the smooth maximum, -1: minimum), and
    each pin's weight over its net's weight sum."""
    if sign > 0:
        ref = np.maximum.reduceat(px, starts)
        w = np.exp((px - ref[net_of_pin]) / gamma)
    else:
        ref = np.minimum.reduceat(px, starts)
        w = np.exp((ref[net_of_pin] - px) / gamma)
    s = np.add.reduceat(w, starts)
    t = np.add.reduceat(px * w, starts)
    return t / s, w / s[net_of_pin]


def wa_wirelength(nl, G, gamma, with_grad=True):
    """WA wirelength per column pair (total and per net) and, if asked, its
    gradient with respect to every instance position ([n_inst, C]).

    Gradient of the smooth maximum with respect to pin i of net e (product
    and quotient rule on the definition):
        d xbar+_e / d x_i = p+_i (1 + (x_i - xbar+_e) / gamma),
        d xbar-_e / d x_i = p-_i (1 - (x_i - xbar-_e) / gamma),
    with p+_i = exp(x_i/gamma) / sum_j exp(x_j/gamma) and p-_i likewise."""
    G = np.asarray(G, np.float64)
    C = G.shape[1]
    net_ptr = nl["net_ptr"].astype(np.int64)
    pin_node = nl["pin_node"].astype(np.int64)
    off = nl["pin_off"].astype(np.float64)
    deg = np.diff(net_ptr)
    nonempty = np.flatnonzero(deg > 0)
    starts = net_ptr[:-1][nonempty]
    # every pin belongs to one net and the nets' pins are consecutive, so the
    # pins in order are the non-empty nets' pins in order
    net_of_pin = np.repeat(np.arange(nonempty.size), deg[nonempty])
    pins = np.arange(net_ptr[-1])
    seg = starts
    per_net = np.zeros((deg.size, C // 2))
    grad = np.zeros((nl["n_inst"], C)) if with_grad else None
    for c in range(C):
        if pins.size == 0:
            continue
        px = G[pin_node[pins], c] + off[pins, c % 2]
        hi, p_hi = _net_means(px, seg, net_of_pin, gamma, +1)
        lo, p_lo = _net_means(px, seg, net_of_pin, gamma, -1)
        per_net[nonempty, c // 2] += hi - lo
        if with_grad:
            gp = p_hi * (1.0 + (px - hi[net_of_pin]) / gamma) - p_lo * (1.0 - (px - lo[net_of_pin]) / gamma)
            np.add.at(grad[:, c], pin_node[pins], gp)
    return per_net.sum(axis=0), per_net, grad
