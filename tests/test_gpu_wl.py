"""GPU parity of the WA wirelength and its gradient (ahr_wl_create /
ahr_wa) against the FP64 oracle, through the C ABI.

Bars (derived from the arithmetic): the device takes every exponential
weight in float32 (relative error below 2^-22 with `expf`), the rest in
float64.  A net's smooth maximum is a weighted mean, so a relative error of
e in every weight moves it by at most e times the net's spread: totals
within 4e-7 relative of the oracle's.  A pin's gradient p (1 +- (x - xbar)/g)
moves by at most a few e times (1 + spread/g); its instance sums a few
pins exactly in 2^-40 fixed point and rounds once to float32: within 2e-6
(1 + |ref|) plus 2^-23 relative."""
import numpy as np
import pytest
import torch

import netlists as H
from oracle import wl_oracle as W
from synth import netlist as N

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2511_10073_amd")

BIG_NETS = N.NetlistConfig("big-nets-30k", 30_000, 60, 200, 31_000, False, 6, 40, 0.30,
                           0.0004, 4500, 6000, 4, 77)
CASES = [("tiny", N.TINY), ("small-movable", N.small(5000, 3, movable_macros=True, ncols=2)),
         ("small-4col", N.small(7000, 4, ncols=4, big_frac=0.01)), ("big-nets", BIG_NETS)]


def check(nl, G, gamma):
    net = A.Netlist(nl)
    wl = A.Wirelength(net)
    try:
        x = torch.as_tensor(G).cuda()
        tot, grad = wl.wa(x, gamma)
        tot2, grad2 = wl.wa(x, gamma)
        only, none = wl.wa(x, gamma, grad=False)
        torch.cuda.synchronize()
    finally:
        wl.close()
    assert none is None
    assert torch.equal(tot, tot2) and torch.equal(grad, grad2) and torch.equal(tot, only)
    # the boundary takes gamma in float32: give the oracle the same value
    rt, _, rg = W.wa_wirelength(nl, G, float(np.float32(gamma)))
    assert np.allclose(tot.cpu().numpy(), rt, rtol=4e-7, atol=0)
    g = grad.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(g - rg) <= 2e-6 * (1 + np.abs(rg)) + 2.0 ** -23 * np.abs(rg)), np.max(np.abs(g - rg))


@pytest.mark.parametrize("name,cfg", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("gamma", [0.5, 8.0])
def test_wa_matches_oracle(name, cfg, gamma):
    nl = N.generate(cfg)
    print(f"[wa] {name}: n_inst={nl['n_inst']} pins={nl['pin_node'].size} gamma={gamma}", flush=True)
    check(nl, nl["g0"], gamma)


@pytest.mark.parametrize("C", [2, 4, 8])
def test_wa_column_counts(C):
    nl = N.generate(N.small(3000, 21, ncols=2))
    rng = np.random.default_rng(C)
    G = np.repeat(nl["g0"], 4, axis=1)[:, :C] + rng.normal(0, 2, (nl["n_inst"], C)).astype(np.float32)
    check(nl, G.astype(np.float32), 1.0)


def test_wa_degenerate_nets():
    # empty, one-pin, repeated-pin and two-pin nets; an instance on no net
    nl = H.make([[], [0], [1, 1], [1, 2], [2, 3, 4, 0]], 6,
                pos=[[0, 0], [1, 5], [4, 2], [-3, 1], [2, -2], [9, 9]])
    check(nl, nl["g0"], 0.7)


def test_wa_full_size_large():
    """large-2.2M (9.45M pins, nets up to ~10k pins), 4 columns, as the benchmark times it."""
    nl = N.generate(N.LARGE)
    print(f"[wa] large: pins={nl['pin_node'].size}", flush=True)
    check(nl, nl["g0"], 4.0)
