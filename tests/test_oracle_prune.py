"""CPU pins of the sparsified signed graph (Section IX, "Further speedups":
keep only the most salient area-hint edges; reading: bin edges whose
salience exp(-maxRatio) |phi_b| falls below prune_tau are left out, macro
edges stay).  A hand-computed window, the unpruned graph filtered edge by
edge, nesting in the threshold, untouched macro edges and the spectral pins
on a pruned graph."""
import math

import numpy as np

import netlists as H
from oracle import ahr_oracle as O
from synth import netlist as N


def bins_of_cell(g, i):
    cols = g.hint_col[g.hint_row_ptr[i]:g.hint_row_ptr[i + 1]]
    return sorted(int(c) - g.first_bvirt for c in cols if c >= g.first_bvirt)


def test_hand_window_saliences():
    """The 4 x 2 scene of the density pins (D = (1, 4, 2, 1, 4, 2, 2, 3)/9,
    mu = 4, C = 1, phi_b = tanh(2 (D_b - 1))) with detection ratio 1, so the
    window is +-2 bins in x and +-1 in y.  Cell c0 at (1, 1), in bin 0, sees
    bins 0, 1, 2, 4, 5, 6 with maxRatio 1/3, 7/3, 13/3, 7/3, 7/3, 13/3 from
    their centres, so saliences e^-maxRatio |phi_b| of 0.676, 0.0780,
    0.0120, 0.0780, 0.0887, 0.0120."""
    flags = [0, 0, 0, 0, H.MACRO, H.FIXED | H.MACRO, H.FIXED]
    sizes = [[1, 1], [2, 1], [3, 1], [4, 1], [4, 2], [1, 1], [0, 0]]
    pos = [[1, 1], [4, 1], [10, 4], [1, 5], [6, 3], [10.5, 1.5], [0, 0]]
    nl = H.make([[0, 1], [2, 3], [1, 2], [0, 6]], 7, flags=flags, sizes=sizes, pos=pos, die=(0, 0, 12, 6))
    for tau, want in [(0.0, [0, 1, 2, 4, 5, 6]), (0.01, [0, 1, 2, 4, 5, 6]), (0.05, [0, 1, 4, 5]),
                      (0.08, [0, 5]), (0.1, [0]), (0.7, [])]:
        p = O.HintParams(nbx=4, nby=2, detection_ratio=1.0, macro_hints=False, prune_tau=tau)
        g = O.build_graph(nl, p, nl["g0"])
        assert bins_of_cell(g, 0) == want, (tau, bins_of_cell(g, 0))
    # the salience figures themselves, from the definitions
    phi = [math.tanh(2 * (a / 9 - 1)) for a in (1, 4, 2, 1, 4, 2, 2, 3)]
    sal = {0: math.exp(-1 / 3) * abs(phi[0]), 1: math.exp(-7 / 3) * abs(phi[1]), 5: math.exp(-7 / 3) * abs(phi[5])}
    assert abs(sal[0] - 0.676) < 1e-3 and abs(sal[1] - 0.0780) < 1e-4 and abs(sal[5] - 0.0887) < 1e-4


def test_pruned_graph_is_the_unpruned_one_filtered_edge_by_edge():
    nl = N.generate(N.small(3000, 41, ncols=2))
    base = O.HintParams(nbx=16, nby=16, detection_ratio=0.2)
    g0 = O.build_graph(nl, base, nl["g0"][:, :2])
    for tau in (0.05, 0.2, 0.5):
        p = O.HintParams(nbx=16, nby=16, detection_ratio=0.2, prune_tau=tau)
        g = O.build_graph(nl, p, nl["g0"][:, :2])
        rows = np.repeat(np.arange(g0.n_tot), np.diff(g0.hint_row_ptr))
        cols = g0.hint_col
        cell = np.where(rows < g0.n_inst, rows, cols)
        binedge = np.maximum(rows, cols) >= g0.first_bvirt
        sal = np.abs(g0.hint_val) / g0.base_weight[cell]
        keep = ~binedge | (sal >= tau)
        near = binedge & (np.abs(sal - tau) <= 1e-12 * tau)
        assert not near.any()                      # no edge sits on the threshold here
        want = set(zip(rows[keep].tolist(), cols[keep].tolist()))
        rows1 = np.repeat(np.arange(g.n_tot), np.diff(g.hint_row_ptr))
        got = set(zip(rows1.tolist(), g.hint_col.tolist()))
        assert got == want
        assert np.array_equal(g.net_q, g0.net_q)
        assert 0 < g.hint_val.size < g0.hint_val.size


def test_thresholds_nest_and_macro_edges_stay():
    nl = N.generate(N.small(2500, 42, ncols=2, movable_macros=True))
    prev = None
    for tau in (0.0, 0.1, 0.3, 0.6, 0.95):
        g = O.build_graph(nl, O.HintParams(nbx=12, nby=12, detection_ratio=0.3, prune_tau=tau), nl["g0"][:, :2])
        rows = np.repeat(np.arange(g.n_tot), np.diff(g.hint_row_ptr))
        edges = set(zip(rows.tolist(), g.hint_col.tolist()))
        macro = {e for e in edges if g.first_mvirt <= max(e) < g.first_bvirt}
        if prev is not None:
            assert edges <= prev[0]
            assert macro == prev[1]
        prev = (edges, macro)


def test_filter_on_pruned_graph_equals_spectral_definition():
    nl = N.generate(N.small(400, 43, ncols=2))
    g = O.build_graph(nl, O.HintParams(nbx=8, nby=8, detection_ratio=0.4, prune_tau=0.3), nl["g0"][:, :2])
    spec = O.FilterSpec(ks=(2, 4, 8), alphas=(0.2, 0.3, 0.5))
    L, T, d, s, lam = O.operator(g)
    ev, U = np.linalg.eigh(L.toarray())
    assert ev.min() >= -1e-12 and ev.max() <= lam + 1e-12
    out, _ = O.apply_filter(nl, g, spec, nl["g0"], return_full=True, pin=False)
    h = sum(a * (1 - ev / lam) ** k for k, a in zip(spec.ks, spec.alphas))
    X = O.expand_signal(nl, g, nl["g0"])
    assert np.max(np.abs(out - U @ (h[:, None] * (U.T @ X)))) <= 1e-11 * np.max(np.abs(X))
