"""GPU parity of GiFt, the GSP-based initializer (Section IV eqs. "GiFt" and
"GiFt filter"), through the C ABI against the FP64 oracle: the netlist graph
without area hints, the three-band bank over two self-loop weights (two
chains added), single-chain banks, fixed rows reset, at small sizes and at
large-2.2M.  Bar: centred relative and per-element error within 1e-5."""
import numpy as np
import pytest
import torch

import gpu_common as U
from oracle import ahr_oracle as O
from synth import netlist as N

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2511_10073_amd")

GRAPH = O.HintParams(expand_macro_pins=False, macro_hints=False, bin_hints=False)
BIG_NETS = N.NetlistConfig("big-nets-30k", 30_000, 60, 200, 31_000, False, 6, 40, 0.30,
                           0.0004, 4500, 6000, 4, 77)
BANKS = {"paper": O.GiftBank(), "one-sigma": O.GiftBank(ks=(2, 4), sigmas=(4.0, 4.0), alphas=(0.4, 0.6)),
         "four": O.GiftBank(ks=(1, 2, 3, 0), sigmas=(0.0, 2.0, 4.0, 1.0), alphas=(0.1, 0.2, 0.3, 0.4))}
CASES = [("tiny", N.TINY), ("small-4col", N.small(7000, 4, ncols=4, big_frac=0.01)), ("big-nets", BIG_NETS)]


def c_bank(bank):
    b = O.GiftBank(tuple(bank.ks), tuple(U.f32(s) for s in bank.sigmas), tuple(U.f32(a) for a in bank.alphas))
    return b, A.gift_spec(b.ks, b.sigmas, b.alphas)


def run(nl, G, bank, expand=False):
    p = O.HintParams(expand_macro_pins=expand, macro_hints=False, bin_hints=False)
    b, cs = c_bank(bank)
    net = A.Netlist(nl)
    x = torch.as_tensor(G).cuda()
    gr = A.Graph(net, U.to_c_params(A, p), x)
    try:
        out = gr.gift(cs, x)
        again = gr.gift(cs, x)
        torch.cuda.synchronize()
        assert torch.equal(out, again)
        out = out.cpu().numpy()
    finally:
        gr.close()
    og = O.build_graph(nl, p, G[:, :2])
    ref = O.gift(nl, og, b, G)
    mov = U.movable_rows(nl)
    err = U.check_filter(out, ref, mov)
    assert np.array_equal(out[~mov], G[~mov])
    return err


@pytest.mark.parametrize("bank", list(BANKS), ids=list(BANKS))
@pytest.mark.parametrize("name,cfg", CASES, ids=[c[0] for c in CASES])
def test_gift_matches_oracle(name, cfg, bank):
    nl = N.generate(cfg)
    G = N.uniform_signal(nl, nl["g0"].shape[1], 1000 + cfg.seed)
    err = run(nl, G, BANKS[bank])
    print(f"[gift] {name} {bank}: rel err {err:.3e}", flush=True)


def test_gift_with_macro_pin_expansion():
    nl = N.generate(N.small(5000, 8, ncols=2))
    G = N.uniform_signal(nl, 2, 8)
    run(nl, G, BANKS["paper"], expand=True)


def test_gift_rejects_a_graph_with_hints():
    nl = N.generate(N.small(500, 9, ncols=2))
    net = A.Netlist(nl)
    x = torch.as_tensor(nl["g0"]).cuda()
    gr = A.Graph(net, U.to_c_params(A, O.HintParams(nbx=8, nby=8)), x)
    try:
        with pytest.raises(A.AhrError) as e:
            gr.gift(A.gift_spec(), x)
        assert e.value.code == A.EINVAL
    finally:
        gr.close()


def test_gift_full_size_large():
    nl = N.generate(N.LARGE)
    G = N.uniform_signal(nl, 4, 1505)
    err = run(nl, G, BANKS["paper"])
    print(f"[gift] large-2.2M: rel err {err:.3e}", flush=True)
