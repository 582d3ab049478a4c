"""Hand-computed pins of the oracle's per-bin, per-row and per-round values.

Each expected value below is worked out by hand from the paper's
definitions (Section V: bin density D_b, baseWeight, the values carried by
the added nodes, and Algorithm 1's per-round rebuild of L_hint), on inputs
small enough to do so, and written in as numbers.  None of them is obtained
by calling the oracle function under test."""
import math

import numpy as np
import pytest

import netlists as H
from oracle import ahr_oracle as O

Q = 2 ** 32


# ------------------------------------------------------- per-bin density D_b

def density_netlist():
    """Die [0, 12] x [0, 6] split 4 x 2 into 3 x 3 bins (b = by * 4 + bx).

    Movable std cells (centre, w x h): c0 (1, 1) 1x1 -> bin 0; c1 (4, 1) 2x1
    -> bin 1; c2 (10, 4) 3x1 -> bin 7; c3 (1, 5) 4x1 -> bin 4.  A movable
    macro m centred (6, 3), 4 x 2, covers [4, 8] x [2, 4]: 2 x 1 in each of
    bins 1, 2, 5, 6.  A fixed macro F centred (10.5, 1.5), 1 x 1, lies in
    bin 3.  A zero-size fixed I/O at (0, 0) adds no area."""
    flags = [0, 0, 0, 0, H.MACRO, H.FIXED | H.MACRO, H.FIXED]
    sizes = [[1, 1], [2, 1], [3, 1], [4, 1], [4, 2], [1, 1], [0, 0]]
    pos = [[1, 1], [4, 1], [10, 4], [1, 5], [6, 3], [10.5, 1.5], [0, 0]]
    nets = [[0, 1], [2, 3], [1, 2], [0, 6]]
    return H.make(nets, 7, flags=flags, sizes=sizes, pos=pos, die=(0, 0, 12, 6))


def test_density_per_bin_on_a_non_square_grid():
    nl = density_netlist()
    p = O.HintParams(nbx=4, nby=2, macro_hints=False)
    g = O.build_graph(nl, p, nl["g0"])
    area = np.array([1, 4, 2, 1, 4, 2, 2, 3], np.float64)     # by hand, bins 0..7
    assert np.allclose(g.density, area / 9.0, rtol=1e-15, atol=0)
    # phi_b = 2 sigmoid(mu (D_b - C)) - 1 with mu = 4, C = 1, per bin
    ref_phi = [2.0 / (1.0 + math.exp(-4.0 * (a / 9.0 - 1.0))) - 1.0 for a in area]
    assert np.allclose(g.phi, ref_phi, rtol=1e-14, atol=0)


def test_density_transposed_grid():
    # the same scene mirrored on the diagonal: 2 x 4 bins of 3 x 3 over [0, 6] x [0, 12]
    nl = density_netlist()
    nl["die"] = np.array([0, 0, 6, 12], np.float32)
    nl["g0"] = nl["g0"][:, ::-1].copy()
    nl["node_size"] = nl["node_size"][:, ::-1].copy()
    g = O.build_graph(nl, O.HintParams(nbx=2, nby=4, macro_hints=False), nl["g0"])
    # bin (bx, by) here is bin (by, bx) above: b' = bx * 2 + by
    area = np.zeros(8)
    for b, a in enumerate([1, 4, 2, 1, 4, 2, 2, 3]):
        bx, by = b % 4, b // 4
        area[bx * 2 + by] = a
    assert np.allclose(g.density, area / 9.0, rtol=1e-15, atol=0)


# ------------------------------------------------------------- baseWeight

def test_base_weight_merges_parallel_edges():
    """Nets [0,1] twice, [0,2,3], [1,4] with weight 3; node 5 is on no net.

    Clique weights w/(p-1): the 2-pin nets give 1 (and 3), the 3-pin net 1/2
    per pair.  Merged rows: 0 -> {1: 2, 2: 1/2, 3: 1/2} (sum 3 over 3
    neighbours), 1 -> {0: 2, 4: 3} (5 over 2), 2 -> {0, 3: 1/2 each},
    3 -> {0, 2: 1/2 each}, 4 -> {1: 3}, 5 -> none."""
    nl = H.make([[0, 1], [0, 1], [0, 2, 3], [1, 4]], 6)
    nl["net_w"] = np.array([1, 1, 1, 3], np.float32)
    g = O.build_graph(nl, O.HintParams(macro_hints=False, bin_hints=False), nl["g0"])
    assert g.qdeg.tolist() == [3 * Q, 5 * Q, Q, Q, 3 * Q, 0]
    assert g.base_weight.tolist() == [1.0, 2.5, 0.5, 0.5, 3.0, 0.0]


# ------------------------------------------------- values of the added nodes

def test_expanded_signal_bins_stars_macros_by_hand():
    """Bin virtual nodes carry the bin centre, a star node the mean of its
    pins (macro pins at macro centre + offset), a macro virtual node its
    macro's centre.  Die [0, 12] x [0, 6], 4 x 2 bins of 3 x 3: centres
    x = 1.5, 4.5, 7.5, 10.5 and y = 1.5 (bins 0..3), 4.5 (bins 4..7)."""
    n = 14
    flags = [0] * 12 + [H.FIXED | H.MACRO, H.MACRO]
    sizes = [[1, 1]] * 12 + [[2, 2], [2, 2]]
    x = np.arange(n, dtype=np.float64)
    pos = np.stack([x, 0.5 * x, -x, 2 * x], axis=1)             # 4 columns: (x, y), (x, y)
    pos[12] = [6.0, 3.0, 5.0, 2.0]                              # fixed macro F
    pos[13] = [9.0, 1.0, 8.0, 4.0]                              # movable macro M
    # net 0: 11 pins on cells 0..10 (a star at clique_max = 10); net 1: 12
    # pins, cells 0..10 and a pin of F at offset (1, -1)
    nets = [list(range(11)), list(range(11)) + [12]]
    off = np.zeros((23, 2), np.float32)
    off[22] = [1.0, -1.0]
    nl = H.make(nets, n, flags=flags, sizes=sizes, pos=pos, die=(0, 0, 12, 6), offsets=off, ncols=4)
    g = O.build_graph(nl, O.HintParams(nbx=4, nby=2), nl["g0"][:, :2])
    assert (g.first_mpin, g.first_star, g.first_mvirt, g.first_bvirt, g.n_tot) == (14, 15, 17, 19, 27)
    X = O.expand_signal(nl, g, nl["g0"])
    # macro pin node: F + (1, -1) in every (x, y) pair
    assert X[14].tolist() == [7.0, 2.0, 6.0, 1.0]
    # star of net 0: mean of cells 0..10 -> x 5, y 2.5, then -5, 10
    assert np.allclose(X[15], [5.0, 2.5, -5.0, 10.0], rtol=1e-15)
    # star of net 1: cells 0..10 (sums 55, 27.5, -55, 110) and the pin node (7, 2, 6, 1), over 12
    assert np.allclose(X[16], [62 / 12, 29.5 / 12, -49 / 12, 111 / 12], rtol=1e-15)
    # macro virtual nodes, in instance order: F then M
    assert X[17].tolist() == [6.0, 3.0, 5.0, 2.0]
    assert X[18].tolist() == [9.0, 1.0, 8.0, 4.0]
    cx = [1.5, 4.5, 7.5, 10.5] * 2
    cy = [1.5] * 4 + [4.5] * 4
    ref = np.stack([cx, cy, cx, cy], axis=1)
    assert np.array_equal(X[19:27], ref)


# ------------------------------------------ Algorithm 1 rebuilds L_hint each round

def test_refine_round_two_uses_the_moved_placement():
    """Two movable cells joined by one 2-pin net, and a pin-less movable
    macro M (centre (0, 0), 2 x 2: footprint [-1, 1]^2) with its virtual node
    v at its centre.  Bins off.  Filter: one power of T with lambda_up = 1,
    so T = D^-1/2 A D^-1/2 on connected rows; gamma = 1, so each round's
    output is the next placement.  All y are 0, so maxRatio = |x|.

    Round 1: cell 0 at x = 0.5 is inside M (edge -exp(-0.5) to v, baseWeight
    1), cell 1 at x = 5 is not.  d0 = 1 + e^-0.5, d1 = 1; v's value is 0, so
      x0' = x1 / sqrt(d0) = 5 / a,  x1' = x0 / sqrt(d0) = 0.5 / a,  a = sqrt(1 + e^-0.5).
    Now cell 1 (x = 0.5/a = 0.393) is inside M and cell 0 (3.93) is not, so
    round 2's operator has the edge (1, v) = -exp(-0.5/a) instead:
      x0'' = x1' / sqrt(1 + e^(-0.5/a)),  x1'' = x0' / sqrt(1 + e^(-0.5/a))."""
    flags = [0, 0, H.MACRO]
    sizes = [[1, 1], [1, 1], [2, 2]]
    pos = [[0.5, 0.0], [5.0, 0.0], [0.0, 0.0]]
    nl = H.make([[0, 1]], 3, flags=flags, sizes=sizes, pos=pos)
    p = O.HintParams(bin_hints=False)
    spec = O.FilterSpec(ks=(1,), alphas=(1.0,), lambda_mode="fixed", lambda_fixed=1.0)
    a = math.sqrt(1 + math.exp(-0.5))
    r1 = O.refine(nl, p, spec, nl["g0"], 1, 1.0)
    assert np.allclose(r1[:, 0], [5 / a, 0.5 / a, 0.0], rtol=1e-7, atol=0)
    b = math.sqrt(1 + math.exp(-0.5 / a))
    r2 = O.refine(nl, p, spec, nl["g0"], 2, 1.0)
    # the hints of round 2 see the round-1 placement in float32 (the signal
    # itself stays float64)
    x1p = float(np.float32(0.5 / a))
    b32 = math.sqrt(1 + math.exp(-x1p))
    assert math.isclose(b, b32, rel_tol=1e-6)
    assert np.allclose(r2[:, 0], [(0.5 / a) / b32, (5 / a) / b32, 0.0], rtol=1e-12, atol=0)
    assert np.all(r2[:, 1] == 0)
    # with round 1's operator kept, round 2 would have given x1'/a, x0'/a
    assert not np.allclose(r2[:2, 0], [(0.5 / a) / a, (5 / a) / a], rtol=1e-3)


@pytest.mark.parametrize("gamma", [0.5])
def test_refine_relaxation_by_hand(gamma):
    """One round with gamma = 0.5 on the scene above: g1 = (g0 + T g0) / 2."""
    flags = [0, 0, H.MACRO]
    nl = H.make([[0, 1]], 3, flags=flags, sizes=[[1, 1], [1, 1], [2, 2]],
                pos=[[0.5, 0.0], [5.0, 0.0], [0.0, 0.0]])
    spec = O.FilterSpec(ks=(1,), alphas=(1.0,), lambda_mode="fixed", lambda_fixed=1.0)
    a = math.sqrt(1 + math.exp(-0.5))
    r = O.refine(nl, O.HintParams(bin_hints=False), spec, nl["g0"], 1, gamma)
    assert np.allclose(r[:, 0], [(0.5 + 5 / a) / 2, (5 + 0.5 / a) / 2, 0.0], rtol=1e-12, atol=0)
