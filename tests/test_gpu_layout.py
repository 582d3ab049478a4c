"""The execution order of the filter: the Hilbert order of the placement or
the netlist's Cuthill-McKee order.  Results do not depend on the order
beyond float32 summation order, so each case checks, under the forced
netlist order, what test_gpu_parity checks under the positions' order
(hint structure exact, filter and refinement within 1e-5 of the oracle);
the default is the positions' order, and the automatic choice keeps it for
the generator's placement and takes the netlist order for uniformly drawn
positions."""
import numpy as np
import pytest
import torch

import gpu_common as U
from netlists import make
from oracle import ahr_oracle as O
from synth import netlist as N

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2511_10073_amd")

BIG_NETS = N.NetlistConfig("big-nets-30k", 30_000, 60, 200, 31_000, False, 6, 40, 0.30,
                           0.0004, 4500, 6000, 4, 77)
CASES = [
    ("tiny", N.TINY, O.HintParams(nbx=8, nby=8)),
    ("small-movable", N.small(5000, 3, movable_macros=True, ncols=2), O.HintParams(nbx=10, nby=10, detection_ratio=0.3)),
    ("small-4col", N.small(7000, 4, ncols=4, big_frac=0.01), O.HintParams(nbx=16, nby=12, detection_ratio=0.2)),
    ("long-rows", BIG_NETS, O.HintParams(nbx=4, nby=4, detection_ratio=0.75)),
]
BANK = U.spec32(O.FilterSpec(ks=(2, 4, 8), alphas=(0.2, 0.3, 0.5)))


def params(A, p, layout):
    c = U.to_c_params(A, p)
    c.flags |= layout
    return c


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def case(request):
    name, cfg, p = request.param
    nl = N.generate(cfg)
    p = U.params32(p)
    print(f"[layout] {name}: n_inst={nl['n_inst']}", flush=True)
    og = O.build_graph(nl, p, nl["g0"][:, :2])
    net = A.Netlist(nl)
    gpos = torch.as_tensor(nl["g0"]).cuda()
    gr = A.Graph(net, params(A, p, A.LAYOUT_NETLIST), gpos)
    yield dict(name=name, nl=nl, p=p, og=og, net=net, gr=gr, gpos=gpos)
    gr.close()


def test_forced_netlist_order_is_used(case):
    assert case["gr"].info()["layout"] == 1


def test_hint_structure_under_netlist_order(case):
    og, ex = case["og"], case["gr"].export()
    assert np.array_equal(ex["net_row_ptr"], og.net_row_ptr.astype(np.int32))
    assert np.array_equal(ex["net_col"], og.net_col.astype(np.int32))
    assert np.array_equal(ex["hint_row_ptr"], og.hint_row_ptr.astype(np.int32))
    r1, c1, v1 = U.sorted_rows(ex["hint_row_ptr"], ex["hint_col"], ex["hint_val"])
    r0, c0, v0 = U.sorted_rows(og.hint_row_ptr, og.hint_col, og.hint_val)
    assert np.array_equal(r1, r0) and np.array_equal(c1, c0)
    assert np.all(np.abs(v1.astype(np.float64) - v0) <= 2.0 ** -22 * np.abs(v0))


def test_filter_and_refine_under_netlist_order(case):
    nl, og, gr, gpos, p = case["nl"], case["og"], case["gr"], case["gpos"], case["p"]
    mov = U.movable_rows(nl)
    ref = O.apply_filter(nl, og, BANK, nl["g0"])
    out = gr.filter(U.to_c_spec(A, BANK), gpos).cpu().numpy()
    err = U.check_filter(out, ref, mov)
    print(f"[{case['name']}] filter rel err {err:.3e}")
    assert np.array_equal(out[~mov], nl["g0"][~mov])
    # two rounds of Algorithm 1 on a fresh graph in the netlist order
    g2 = A.Graph(case["net"], params(A, p, A.LAYOUT_NETLIST), None)
    try:
        got = g2.refine(U.to_c_spec(A, BANK), gpos, 2, 0.5).cpu().numpy()
        assert g2.info()["layout"] == 1
    finally:
        g2.close()
    want = O.refine(nl, p, BANK, nl["g0"], 2, 0.5)
    err = U.check_filter(got, want, mov)
    print(f"[{case['name']}] refine rel err {err:.3e}")


def test_filter_same_bits_across_calls_under_netlist_order(case):
    gr, gpos = case["gr"], case["gpos"]
    a = gr.filter(U.to_c_spec(A, BANK), gpos)
    b = gr.filter(U.to_c_spec(A, BANK), gpos)
    assert torch.equal(a, b)


def components():
    """Two rings, a path, a 14-pin net (a star: no instance-to-instance
    edge) and isolated cells: the netlist order reaches one component from
    its start and appends the other instances in id order."""
    nets = [[i, (i + 1) % 10] for i in range(10)] + [[10 + i, 10 + (i + 1) % 10] for i in range(10)]
    nets += [[20 + i, 21 + i] for i in range(5)] + [list(range(26, 40))]
    return make(nets, 45, ncols=4)


@pytest.mark.parametrize("which", ["components", "no-nets", "one-instance"])
def test_netlist_order_on_degenerate_netlists(which):
    nl = {"components": components, "no-nets": lambda: make([], 30, ncols=4),
          "one-instance": lambda: make([[0]], 1, ncols=2)}[which]()
    p = U.params32(O.HintParams(nbx=3, nby=3, detection_ratio=0.5))
    og = O.build_graph(nl, p, nl["g0"][:, :2])
    net = A.Netlist(nl)
    x = torch.as_tensor(nl["g0"]).cuda()
    gr = A.Graph(net, params(A, p, A.LAYOUT_NETLIST), x)
    try:
        assert gr.info()["layout"] == 1
        ex = gr.export()
        assert np.array_equal(ex["net_row_ptr"], og.net_row_ptr.astype(np.int32))
        assert np.array_equal(ex["hint_row_ptr"], og.hint_row_ptr.astype(np.int32))
        out = gr.filter(U.to_c_spec(A, BANK), x).cpu().numpy()
        again = gr.filter(U.to_c_spec(A, BANK), x).cpu().numpy()
    finally:
        gr.close()
    assert np.array_equal(out, again)
    mov = U.movable_rows(nl)
    assert np.array_equal(out[~mov], nl["g0"][~mov])
    ref = np.asarray(O.apply_filter(nl, og, BANK, nl["g0"]), np.float64)
    if np.linalg.norm(ref[mov] - ref[mov].mean(axis=0)) == 0:      # one row: no centred scale
        assert np.allclose(out[mov], ref[mov], rtol=1e-6, atol=1e-6)
    else:
        err = U.check_filter(out, ref, mov)
        print(f"[{which}] filter rel err {err:.3e}")


def test_automatic_choice():
    nl = N.generate(N.small(20000, 62, ncols=4))
    net = A.Netlist(nl)
    p = U.to_c_params(A, O.HintParams(nbx=16, nby=16, detection_ratio=0.2))
    g0 = torch.as_tensor(nl["g0"]).cuda()
    u = torch.as_tensor(N.uniform_signal(nl, 4, 7)).cuda()
    for pos in (g0, u):                           # by default the Hilbert order, whatever the positions
        g = A.Graph(net, p, pos)
        try:
            assert g.info()["layout"] == 0
        finally:
            g.close()
    p.flags |= A.LAYOUT_AUTO
    g = A.Graph(net, p, g0)
    try:
        assert g.info()["layout"] == 0            # the generator's placement follows its netlist
    finally:
        g.close()
    g = A.Graph(net, p, u)
    try:
        assert g.info()["layout"] == 1            # uniform positions say nothing about the netlist
    finally:
        g.close()


def test_hop_shape_follows_locality():
    """Under AHR_HOP_AUTO (the default) a graph whose execution order is
    local runs the 4-lane hop, one whose order has no locality (uniformly
    drawn positions) the row-block hop; either way the filter is the
    oracle's within 1e-5."""
    nl = N.generate(N.small(20000, 62, ncols=4))
    net = A.Netlist(nl)
    p = U.params32(O.HintParams(nbx=16, nby=16, detection_ratio=0.2))
    mov = U.movable_rows(nl)
    assert A.filter_get_tune()[0] == A.HOP_AUTO
    u = N.uniform_signal(nl, 4, 7)
    for pos, lanes in ((nl["g0"], 4), (u, A.HOP_ROW_BLOCK)):
        g = A.Graph(net, U.to_c_params(A, p), torch.as_tensor(pos).cuda())
        try:
            assert g.info()["hop_lanes"] == 0              # read with the first normalisation
            out = g.filter(U.to_c_spec(A, BANK), torch.as_tensor(pos).cuda()).cpu().numpy()
            assert g.info()["hop_lanes"] == lanes
        finally:
            g.close()
        og = O.build_graph(nl, p, pos[:, :2])
        err = U.check_filter(out, O.apply_filter(nl, og, BANK, pos), mov)
        print(f"[hop shape {lanes}] filter rel err {err:.3e}")


def test_conflicting_layout_flags_rejected():
    nl = N.generate(N.TINY)
    net = A.Netlist(nl)
    p = U.to_c_params(A, O.HintParams(nbx=8, nby=8))
    p.flags |= A.LAYOUT_AUTO | A.LAYOUT_NETLIST
    with pytest.raises(Exception, match="exclude each other"):
        A.Graph(net, p, torch.as_tensor(nl["g0"]).cuda())
