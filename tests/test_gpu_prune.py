"""GPU parity of the sparsified signed graph (salience pruning of the bin
hint edges, prune_tau > 0) through the C ABI against the FP64 oracle: the
hint structure exact and its weights within float32 rounding, the filter
and Algorithm 1 within the FP32 bound (centred and per element), at small
sizes and at the full mid-210k and large-2.2M workloads, for windows of up
to 64 slots (pruning decided in the count pass) and wider ones (pruned
entries compacted after the fill)."""
import numpy as np
import pytest
import torch

import gpu_common as U
from oracle import ahr_oracle as O
from synth import netlist as N

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2511_10073_amd")

BANK = O.FilterSpec(ks=(2, 4, 8), alphas=(0.2, 0.3, 0.5))
BIG_NETS = N.NetlistConfig("big-nets-30k", 30_000, 60, 200, 31_000, False, 6, 40, 0.30,
                           0.0004, 4500, 6000, 4, 77)
CASES = [
    ("small-movable", N.small(5000, 3, movable_macros=True, ncols=2), dict(nbx=10, nby=10, detection_ratio=0.3)),
    ("small-4col", N.small(7000, 4, ncols=4, big_frac=0.01), dict(nbx=16, nby=12, detection_ratio=0.2)),
    ("long-rows", BIG_NETS, dict(nbx=4, nby=4, detection_ratio=0.75)),
    # a 7 x 9 window (63 slots, the pruning decided in the count pass with the
    # mask's high bits in use) and a 9 x 9 one (81 slots: holes and compaction)
    ("window-63", N.small(5000, 3, ncols=2), dict(nbx=12, nby=16, detection_ratio=0.5)),
    ("window-81", N.small(5000, 3, ncols=2), dict(nbx=16, nby=16, detection_ratio=0.6)),
]


def hint_entries(rp, col, val):
    rows = np.repeat(np.arange(rp.size - 1), np.diff(rp))
    o = np.lexsort((col, rows))
    return rows[o], np.asarray(col)[o], np.asarray(val, np.float64)[o]


def check_graph_and_filter(nl, p, spec):
    net = A.Netlist(nl)
    x = torch.as_tensor(nl["g0"]).cuda()
    gr = A.Graph(net, U.to_c_params(A, p), x)
    try:
        out = gr.filter(U.to_c_spec(A, spec), x).cpu().numpy()
        ex = gr.export()
    finally:
        gr.close()
    og = O.build_graph(nl, p, nl["g0"][:, :2])
    assert np.array_equal(ex["hint_row_ptr"], og.hint_row_ptr.astype(np.int32))
    r1, c1, v1 = hint_entries(ex["hint_row_ptr"], ex["hint_col"], ex["hint_val"])
    r0, c0, v0 = hint_entries(og.hint_row_ptr, og.hint_col, og.hint_val)
    assert np.array_equal(r1, r0) and np.array_equal(c1, c0)
    assert np.all(np.abs(v1 - v0) <= 2.0 ** -22 * np.abs(v0))
    ref = O.apply_filter(nl, og, spec, nl["g0"])
    err = U.check_filter(out, ref, U.movable_rows(nl))
    return og, err


@pytest.mark.parametrize("tau", [0.05, 0.3])
@pytest.mark.parametrize("name,cfg,kw", CASES, ids=[c[0] for c in CASES])
def test_pruned_graph_and_filter_match_oracle(name, cfg, kw, tau):
    nl = N.generate(cfg)
    p = U.params32(O.HintParams(prune_tau=tau, **kw))
    full = U.params32(O.HintParams(**kw))
    og, err = check_graph_and_filter(nl, p, U.spec32(BANK))
    n_full = O.build_graph(nl, full, nl["g0"][:, :2]).hint_val.size
    print(f"[prune] {name} tau={tau}: {og.hint_val.size} of {n_full} hint entries, rel err {err:.3e}", flush=True)
    assert og.hint_val.size < n_full


def test_pruned_refine_round_by_round():
    nl = N.generate(N.small(7000, 4, ncols=4, big_frac=0.01))
    p = U.params32(O.HintParams(nbx=16, nby=12, detection_ratio=0.2, prune_tau=0.2))
    spec = U.spec32(BANK)
    cs = U.to_c_spec(A, spec)
    net = A.Netlist(nl)
    x = torch.as_tensor(nl["g0"]).cuda()
    gr = A.Graph(net, U.to_c_params(A, p), x)
    try:
        cur = x
        for r in range(3):
            nxt = gr.refine(cs, cur, 1, 0.5)
            ref = O.refine(nl, p, spec, cur.cpu().numpy(), 1, 0.5)
            U.check_filter(nxt.cpu().numpy(), ref, U.movable_rows(nl))
            cur = nxt
    finally:
        gr.close()


@pytest.mark.parametrize("cfg_name", ["MID", "LARGE"])
def test_pruned_full_size(cfg_name):
    cfg = getattr(N, cfg_name)
    nl = N.generate(cfg)
    p = U.params32(O.HintParams(nbx=32, nby=32, prune_tau=0.1))
    og, err = check_graph_and_filter(nl, p, U.spec32(BANK))
    print(f"[prune] {cfg.name} tau=0.1: {og.hint_val.size} hint entries, rel err {err:.3e}", flush=True)
