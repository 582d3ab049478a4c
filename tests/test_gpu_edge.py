"""GPU parity on degenerate inputs, through the C ABI against the FP64
oracle:

- a netlist without nets (every row isolated);
- empty and single-pin nets;
- a net listing one cell twice, and a net whose pins are all one cell;
- non-uniform net weights;
- every net a star;
- hints switched off;
- a single instance;
- lambda_up fixed at 0 (T = I);
- a very high filter order;
- a graph built with no placement, its sizes and CSR read before any hints.

Bars as in the main parity tests: CSR bit-exact, filter within 1e-5
centred relative error (exact where the result is an identity), fixed
rows equal to their input."""
import numpy as np
import pytest
import torch

import gpu_common as U
from netlists import make
from oracle import ahr_oracle as O
from synth import netlist as N

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2511_10073_amd")

FILTER_TOL = 1e-5


def run_case(nl, p, spec, check_csr=True):
    p = U.params32(p)
    spec = U.spec32(spec)
    og = O.build_graph(nl, p, nl["g0"][:, :2])
    net = A.Netlist(nl)
    x = torch.as_tensor(nl["g0"]).cuda()
    gr = A.Graph(net, U.to_c_params(A, p), x)
    try:
        if check_csr:
            ex = gr.export()
            assert np.array_equal(ex["net_row_ptr"], og.net_row_ptr.astype(np.int32))
            assert np.array_equal(ex["net_col"], og.net_col.astype(np.int32))
            assert np.array_equal(ex["net_q"], og.net_q)
        out = gr.filter(U.to_c_spec(A, spec), x).cpu().numpy()
        ref = O.apply_filter(nl, og, spec, nl["g0"])
        hp = gr.hpwl(x).cpu().numpy()
        ref_hp, _ = O.hpwl(nl, nl["g0"])
    finally:
        gr.close()
    mov = U.movable_rows(nl)
    assert np.array_equal(out[~mov], nl["g0"][~mov])
    assert np.allclose(hp, ref_hp, rtol=1e-12, atol=1e-12)
    return out, ref, mov


def check_close(out, ref, mov):
    ref = np.asarray(ref, np.float64)
    if np.linalg.norm(ref[mov] - ref[mov].mean(axis=0)) == 0:
        assert np.allclose(out[mov], ref[mov], rtol=1e-6, atol=1e-6)
    else:
        U.check_filter(out, ref, mov)


BANK = O.FilterSpec(ks=(2, 4, 8), alphas=(0.2, 0.3, 0.5))


def test_no_nets_every_row_isolated():
    nl = make([], 40, ncols=4)
    out, ref, mov = run_case(nl, O.HintParams(nbx=4, nby=4), BANK)
    # isolated rows are identity rows of every power: out = (sum alpha) x
    assert np.allclose(out[mov], np.float32(1.0) * nl["g0"][mov], rtol=1e-6)
    check_close(out, ref, mov)


def test_empty_and_single_pin_nets():
    nets = [[], [3], [0, 1], [], [2, 5, 7], [4], [6, 1, 0, 8]]
    nl = make(nets, 12, ncols=2)
    out, ref, mov = run_case(nl, O.HintParams(nbx=3, nby=3, detection_ratio=0.5), BANK)
    check_close(out, ref, mov)


def test_repeated_pins_and_one_cell_net():
    nets = [[0, 1, 0, 2], [3, 3, 3], [4, 5, 6, 4, 5], [7, 8], [8, 9, 7]]
    nl = make(nets, 10, ncols=2)
    out, ref, mov = run_case(nl, O.HintParams(nbx=2, nby=2), O.FilterSpec(ks=(3,), alphas=(1.0,)))
    check_close(out, ref, mov)


def test_net_weights():
    rng = np.random.default_rng(5)
    nets = [list(rng.choice(30, rng.integers(2, 14), replace=False)) for _ in range(45)]
    nl = make(nets, 30, ncols=4)
    nl["net_w"] = rng.uniform(0.1, 3.0, len(nets)).astype(np.float32)
    out, ref, mov = run_case(nl, O.HintParams(nbx=4, nby=4, detection_ratio=0.5, clique_max=6), BANK)
    check_close(out, ref, mov)


def test_every_net_a_star():
    rng = np.random.default_rng(6)
    nets = [list(rng.choice(60, rng.integers(2, 9), replace=False)) for _ in range(70)]
    nl = make(nets, 60, ncols=2)
    out, ref, mov = run_case(nl, O.HintParams(nbx=4, nby=4, clique_max=1), BANK)
    check_close(out, ref, mov)


@pytest.mark.parametrize("hints", ["none", "pins-only", "macros-only", "bins-only"])
def test_hint_switches(hints):
    rng = np.random.default_rng(7)
    n = 300
    flags = np.zeros(n, np.uint8)
    sizes = np.ones((n, 2), np.float32)
    flags[:4] = 3                       # fixed macros
    sizes[:4] = 4.0
    pos = rng.uniform(-9, 9, (n, 2)).astype(np.float32)
    nets = [list(rng.choice(n, rng.integers(2, 6), replace=False)) for _ in range(320)]
    offsets = rng.uniform(-1, 1, (sum(len(e) for e in nets), 2)).astype(np.float32)
    nl = make(nets, n, flags=flags, sizes=sizes, pos=pos, offsets=offsets)
    kw = dict(none=dict(expand_macro_pins=False, macro_hints=False, bin_hints=False),
              **{"pins-only": dict(macro_hints=False, bin_hints=False),
                 "macros-only": dict(bin_hints=False),
                 "bins-only": dict(macro_hints=False)})[hints]
    out, ref, mov = run_case(nl, O.HintParams(nbx=5, nby=5, detection_ratio=0.4, **kw), BANK)
    check_close(out, ref, mov)


def test_single_instance():
    nl = make([[0]], 1, ncols=2)
    out, ref, mov = run_case(nl, O.HintParams(nbx=1, nby=1), BANK)
    check_close(out, ref, mov)


def test_fixed_lambda_zero_is_identity():
    rng = np.random.default_rng(8)
    nets = [list(rng.choice(50, 3, replace=False)) for _ in range(60)]
    nl = make(nets, 50, ncols=2)
    spec = O.FilterSpec(ks=(1, 3), alphas=(0.5, 0.25), lambda_mode="fixed", lambda_fixed=0.0)
    out, ref, mov = run_case(nl, O.HintParams(nbx=3, nby=3), spec)
    assert np.allclose(out[mov], 0.75 * nl["g0"][mov], rtol=1e-6)
    check_close(out, ref, mov)


def test_high_order():
    rng = np.random.default_rng(9)
    nets = [list(rng.choice(400, rng.integers(2, 8), replace=False)) for _ in range(420)]
    nl = make(nets, 400, ncols=4)
    out, ref, mov = run_case(nl, O.HintParams(nbx=6, nby=6, detection_ratio=0.3),
                             O.FilterSpec(ks=(16, 64), alphas=(0.5, 0.5)))
    check_close(out, ref, mov)


def test_graph_without_placement_then_hints():
    """A graph built with no placement holds only the netlist part: its sizes
    and exported CSR are read from the in-place merged rows (no hints, no
    execution layout yet).  Hints added afterwards give the same graph as a
    build with the placement."""
    nl = N.generate(N.TINY)
    p = U.params32(O.HintParams(nbx=8, nby=8))
    og = O.build_graph(nl, p, nl["g0"][:, :2])
    net = A.Netlist(nl)
    x = torch.as_tensor(nl["g0"]).cuda()
    gr = A.Graph(net, U.to_c_params(A, p), None)
    try:
        inf = gr.info()
        assert inf["nnz_net"] == og.net_col.size and inf["nnz_hint"] == 0
        ex = gr.export()
        assert np.array_equal(ex["net_row_ptr"], og.net_row_ptr.astype(np.int32))
        assert np.array_equal(ex["net_col"], og.net_col.astype(np.int32))
        assert np.array_equal(ex["net_q"], og.net_q)
        gr.update_hints(x)
        inf = gr.info()
        assert inf["nnz_net"] == og.net_col.size and inf["nnz_hint"] == og.hint_col.size
        ex = gr.export()
        assert np.array_equal(ex["hint_row_ptr"], og.hint_row_ptr.astype(np.int32))
        spec = U.spec32(BANK)
        out = gr.filter(U.to_c_spec(A, spec), x).cpu().numpy()
    finally:
        gr.close()
    ref = O.apply_filter(nl, og, spec, nl["g0"])
    check_close(out, ref, U.movable_rows(nl))
