"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element
by element, on seeded inputs that span several tiles and ragged tails.

Bars: netlist CSR (row pointers, columns, integer weights) bit-exact; hint
structure (rows, columns) exact and weights within float32 rounding of the
float64 values; the filter within 1e-5 centred relative error of the oracle
(the FP32 bound); HPWL within 1e-9 relative (both float64)."""
import numpy as np
import pytest
import torch

import gpu_common as U
from oracle import ahr_oracle as O
from synth import netlist as N

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2511_10073_amd")

FILTER_TOL = 1e-5

BIG_NETS = N.NetlistConfig("big-nets-30k", 30_000, 60, 200, 31_000, False, 6, 40, 0.30,
                           0.0004, 4500, 6000, 4, 77)

CASES = [
    ("tiny", N.TINY, O.HintParams(nbx=8, nby=8)),
    ("small-movable", N.small(5000, 3, movable_macros=True, ncols=2), O.HintParams(nbx=10, nby=10, detection_ratio=0.3)),
    ("small-4col", N.small(7000, 4, ncols=4, big_frac=0.01), O.HintParams(nbx=16, nby=12, detection_ratio=0.2)),
    ("long-rows", BIG_NETS, O.HintParams(nbx=4, nby=4, detection_ratio=0.75)),
]


def device_setup(nl, p, g=None):
    net = A.Netlist(nl)
    gpos = torch.as_tensor(nl["g0"] if g is None else g).cuda()
    gr = A.Graph(net, U.to_c_params(A, p), gpos)
    return net, gr, gpos


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def case(request):
    name, cfg, p = request.param
    nl = N.generate(cfg)
    p = U.params32(p)
    print(f"[case] {name}: n_inst={nl['n_inst']} nets={nl['net_ptr'].size - 1}", flush=True)
    og = O.build_graph(nl, p, nl["g0"][:, :2])
    net, gr, gpos = device_setup(nl, p)
    yield dict(name=name, nl=nl, p=p, og=og, net=net, gr=gr, gpos=gpos)
    gr.close()


def test_node_ranges(case):
    og, inf = case["og"], case["gr"].info()
    assert (inf["n_inst"], inf["n_tot"], inf["first_mpin"], inf["first_star"], inf["first_mvirt"],
            inf["first_bvirt"]) == (og.n_inst, og.n_tot, og.first_mpin, og.first_star, og.first_mvirt,
                                    og.first_bvirt)


def test_netlist_csr_bit_exact(case):
    og, ex = case["og"], case["gr"].export()
    assert np.array_equal(ex["net_row_ptr"], og.net_row_ptr.astype(np.int32))
    assert np.array_equal(ex["net_col"], og.net_col.astype(np.int32))
    assert np.array_equal(ex["net_q"], og.net_q)


def test_hint_structure_exact_and_weights(case):
    og, ex = case["og"], case["gr"].export()
    assert np.array_equal(ex["hint_row_ptr"], og.hint_row_ptr.astype(np.int32))
    r1, c1, v1 = U.sorted_rows(ex["hint_row_ptr"], ex["hint_col"], ex["hint_val"])
    r0, c0, v0 = U.sorted_rows(og.hint_row_ptr, og.hint_col, og.hint_val)
    assert np.array_equal(r1, r0) and np.array_equal(c1, c0)
    # float32 storage of float64 weights: within one float32 rounding (+ exp's last bits)
    d = np.abs(v1.astype(np.float64) - v0)
    bad = d > 2.0 ** -22 * np.abs(v0)
    if bad.any():
        k = np.flatnonzero(bad)[:10]
        print("worst:", list(zip(r0[k], c0[k], v0[k], v1[k])))
        print("phi near the failing bins:", og.phi[np.clip(c0[k] - og.first_bvirt, 0, og.phi.size - 1)])
    assert not bad.any()


@pytest.mark.parametrize("spec", [
    O.FilterSpec(ks=(4,), alphas=(1.0,)),
    O.FilterSpec(ks=(2, 4, 8), alphas=(0.2, 0.3, 0.5)),
    O.FilterSpec(ks=(3, 5), alphas=(0.5, 0.5), sigma=0.5),
    O.FilterSpec(ks=(1,), alphas=(1.0,), lambda_mode="fixed", lambda_fixed=1.0),
    O.FilterSpec(ks=(0, 2), alphas=(0.25, 0.75)),
], ids=["k4", "bank248", "sigma", "fixed1", "k0"])
def test_filter_matches_oracle(case, spec):
    nl, og, gr, gpos = case["nl"], case["og"], case["gr"], case["gpos"]
    spec = U.spec32(spec)
    ref, lam = O.apply_filter(nl, og, spec, nl["g0"], return_full=True)
    out = gr.filter(U.to_c_spec(A, spec), gpos).cpu().numpy()
    ex = gr.export()
    L, T, d, s, lam0 = O.operator(og, spec.sigma, spec.lambda_mode, spec.lambda_fixed)
    assert abs(ex["lambda_up"] - lam0) <= 1e-6 * lam0
    assert np.allclose(ex["degree"], d, rtol=1e-6, atol=0)
    mov = U.movable_rows(nl)
    err = U.check_filter(out, ref[:og.n_inst], mov)
    print(f"[{case['name']}] rel err {err:.3e}")
    assert err <= FILTER_TOL
    fixed = ~mov
    assert np.array_equal(out[fixed], nl["g0"][fixed])


def test_filter_other_column_counts(case):
    nl, og, gr = case["nl"], case["og"], case["gr"]
    spec = U.spec32(O.FilterSpec(ks=(2, 4, 8), alphas=(0.2, 0.3, 0.5)))
    for C in (1, 2, 4, 8):
        rng = np.random.default_rng(C)
        G = np.repeat(nl["g0"][:, :2], 4, axis=1)[:, :C].copy()
        mov = U.movable_rows(nl)
        G[mov] += rng.normal(0, 1, (mov.sum(), C)).astype(np.float32)
        ref = O.apply_filter(nl, og, spec, G)
        out = gr.filter(U.to_c_spec(A, spec), torch.as_tensor(G).cuda()).cpu().numpy()
        U.check_filter(out, ref, mov)


def test_filter_is_deterministic(case):
    gr, gpos = case["gr"], case["gpos"]
    spec = U.to_c_spec(A, O.FilterSpec(ks=(2, 4, 8), alphas=(0.2, 0.3, 0.5)))
    a = gr.filter(spec, gpos).cpu().numpy()
    gr.update_hints(gpos)
    b = gr.filter(spec, gpos).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("lanes", [1, 8, 64, "row-block"])
def test_hop_forms_match_oracle(case, lanes):
    """Every launch form of the hop (lanes per row, or the LDS-staged row
    blocks) gives the oracle's filter within the FP32 bound, deterministically."""
    nl, og, gr = case["nl"], case["og"], case["gr"]
    saved = A.filter_get_tune()
    A.filter_tune(A.HOP_ROW_BLOCK if lanes == "row-block" else lanes, -1)
    try:
        spec = U.spec32(O.FilterSpec(ks=(2, 4, 8), alphas=(0.2, 0.3, 0.5)))
        mov = U.movable_rows(nl)
        for C in (1, 4, 8):
            G = np.repeat(nl["g0"][:, :2], 4, axis=1)[:, :C].copy()
            G[mov] += np.random.default_rng(C).normal(0, 1, (mov.sum(), C)).astype(np.float32)
            ref = O.apply_filter(nl, og, spec, G)
            x = torch.as_tensor(G).cuda()
            out = gr.filter(U.to_c_spec(A, spec), x)
            again = gr.filter(U.to_c_spec(A, spec), x)
            assert torch.equal(out, again)
            U.check_filter(out.cpu().numpy(), ref, mov)
    finally:
        A.filter_tune(*saved)


def test_hpwl_matches_oracle(case):
    nl, gr, gpos = case["nl"], case["gr"], case["gpos"]
    C = gpos.shape[1]
    ref, _ = O.hpwl(nl, nl["g0"])
    got = gr.hpwl(gpos).cpu().numpy()
    assert got.shape == (C // 2,)
    assert np.allclose(got, ref, rtol=1e-12, atol=0)


def test_refine_round_by_round(case):
    """Algorithm 1: every round's structure is decided on the GPU's own
    float32 placement, so the oracle is fed the same placement per round."""
    nl, p, gr, gpos = case["nl"], case["p"], case["gr"], case["gpos"]
    spec = U.spec32(O.FilterSpec(ks=(2, 4, 8), alphas=(0.2, 0.3, 0.5)))
    cs = U.to_c_spec(A, spec)
    gamma = 0.5
    cur = gpos.clone()
    mov = U.movable_rows(nl)
    fixed = ~mov
    for r in range(3):
        nxt = gr.refine(cs, cur, 1, gamma)
        G = cur.cpu().numpy()
        ref = O.refine(nl, p, spec, G, 1, gamma)
        got = nxt.cpu().numpy()
        # compare the filtered part: (got - (1-gamma) G) / gamma against the oracle's
        U.check_filter(got, ref, mov)
        assert np.array_equal(got[fixed], G[fixed])
        cur = nxt
    full = gr.refine(cs, gpos, 3, gamma).cpu().numpy()
    assert np.array_equal(full.view(np.uint32), cur.cpu().numpy().view(np.uint32))


@pytest.mark.parametrize("name", ["small-4col", "long-rows"])
def test_first_hop_bound_same_bits(name):
    """The first filter on new hints forms lambda_up inside its first hop;
    a second filter on the same graph uses the bound already formed by it
    and the plain first hop.  Both outputs and lambda_up must agree bit for
    bit, and match the oracle."""
    cfg, p = {c[0]: (c[1], c[2]) for c in CASES}[name]
    nl = N.generate(cfg)
    p = U.params32(p)
    spec = U.spec32(O.FilterSpec(ks=(2, 4, 8), alphas=(0.2, 0.3, 0.5)))
    cs = U.to_c_spec(A, spec)
    saved = A.filter_get_tune()
    A.filter_tune(4, -1)
    net, gr, gpos = device_setup(nl, p)
    try:
        y1 = gr.filter(cs, gpos).clone()
        lam1 = gr.export()["lambda_up"]
        y2 = gr.filter(cs, gpos)
        lam2 = gr.export()["lambda_up"]
        assert lam1 == lam2
        assert torch.equal(y1, y2)
        og = O.build_graph(nl, p, nl["g0"][:, :2])
        ref = O.apply_filter(nl, og, spec, nl["g0"])
        U.check_filter(y1.cpu().numpy(), ref, U.movable_rows(nl))
    finally:
        gr.close()
        A.filter_tune(*saved)
