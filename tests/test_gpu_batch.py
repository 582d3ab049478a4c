"""GPU: the batched filter (many netlists as one block-diagonal operator,
HIP-graph replays, tuned launch shape) through the C ABI.

Bars: every member's slice of the batched output is bit-identical to the
single-graph filter on that member for the same lanes per row (any column
tile), and within the FP32 bound (1e-5 centred relative error) of the FP64
oracle; every HIP-graph replay equals the directly launched result."""
import numpy as np
import pytest
import torch

import gpu_common as U
from oracle import ahr_oracle as O
from synth import netlist as N

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2511_10073_amd")

FILTER_TOL = 1e-5

# uneven members: long rows (150-pin stars, crowded bins), movable macros,
# a member smaller than one workgroup of rows, different bin grids
MEMBERS = [
    (N.small(600, 11, ncols=4), O.HintParams(nbx=6, nby=6)),
    (N.small(3000, 12, ncols=4, big_frac=0.01), O.HintParams(nbx=8, nby=8, detection_ratio=0.3)),
    (N.small(150, 13, ncols=4, n_macro=2), O.HintParams(nbx=4, nby=4)),
    (N.batch_member(9000, 14, 0.03), O.HintParams(nbx=16, nby=16, detection_ratio=0.2)),
    (N.small(1200, 15, ncols=4, movable_macros=True), O.HintParams(nbx=10, nby=7)),
]

BANK = O.FilterSpec(ks=(2, 4, 8), alphas=(0.2, 0.3, 0.5))
SPECS = {
    "bank248": BANK,
    "k4": O.FilterSpec(ks=(4,), alphas=(1.0,)),
    "sigma": O.FilterSpec(ks=(3,), alphas=(1.0,), sigma=0.5),
    "fixed-lambda-band0": O.FilterSpec(ks=(0, 5), alphas=(0.25, 0.75), lambda_mode="fixed", lambda_fixed=2.5),
    "k0": O.FilterSpec(ks=(0,), alphas=(1.0,)),
}


@pytest.fixture(scope="module")
def batch():
    nls = [N.generate(cfg) for cfg, _ in MEMBERS]
    ps = [U.params32(p) for _, p in MEMBERS]
    print("[batch] members:", [int(nl["n_inst"]) for nl in nls], flush=True)
    nets = [A.Netlist(nl) for nl in nls]
    pos = torch.as_tensor(np.concatenate([nl["g0"] for nl in nls])).cuda()
    b = A.Batch(nets, [U.to_c_params(A, p) for p in ps], pos)
    graphs = [A.Graph(net, U.to_c_params(A, p), torch.as_tensor(nl["g0"]).cuda())
              for net, nl, p in zip(nets, nls, ps)]
    saved = A.filter_get_tune()
    yield dict(nls=nls, ps=ps, nets=nets, pos=pos, b=b, graphs=graphs)
    A.filter_tune(*saved)
    for g in graphs:
        g.close()
    b.close()


def signal(bt, C):
    """A C-column signal: the placement's columns, repeated for C = 8."""
    x = bt["pos"] if C == 4 else (bt["pos"][:, :2] if C == 2 else torch.cat([bt["pos"], bt["pos"] * 0.5], 1))
    return x.contiguous()


def members_alone(bt, spec, x):
    outs = []
    for g, lo, hi in zip(bt["graphs"], bt["b"].offsets[:-1], bt["b"].offsets[1:]):
        outs.append(g.filter(spec, x[lo:hi].contiguous()))
    return torch.cat(outs)


def test_info(batch):
    inf = batch["b"].info()
    ginf = [g.info() for g in batch["graphs"]]
    assert inf["n_graphs"] == len(MEMBERS)
    assert inf["n_inst"] == sum(i["n_inst"] for i in ginf)
    assert inf["n_tot"] == sum(i["n_tot"] for i in ginf)
    assert inf["nnz_net"] == sum(i["nnz_net"] for i in ginf)
    assert inf["nnz_hint"] == sum(i["nnz_hint"] for i in ginf)
    assert inf["n_long_rows"] > 0


@pytest.mark.parametrize("C", [2, 4, 8])
@pytest.mark.parametrize("lanes", [1, 2, 4, 16, 64, "row-block"])
def test_batched_equals_members_bit_exact(batch, C, lanes):
    b = batch["b"]
    lanes = A.HOP_ROW_BLOCK if lanes == "row-block" else lanes
    spec = U.to_c_spec(A, BANK)
    x = signal(batch, C)
    A.filter_tune(lanes, -1)
    ref = members_alone(batch, spec, x)
    for ct in [t for t in (8, 4, 2, 1) if t <= C]:
        b.set_config(C, lanes, ct)
        assert b.get_config(C) == (lanes, ct)
        y = b.filter(spec, x)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), f"lanes {lanes} tile {ct}: max |diff| {float((y - ref).abs().max())}"


@pytest.mark.parametrize("name", list(SPECS))
def test_specs_bit_exact_and_oracle(batch, name):
    b = batch["b"]
    so = U.spec32(SPECS[name])
    spec = U.to_c_spec(A, so)
    x = signal(batch, 4)
    A.filter_tune(2, -1)
    b.set_config(4, 2, 2)
    y = b.filter(spec, x)
    ref = members_alone(batch, spec, x)
    assert torch.equal(y, ref)
    y = y.cpu().numpy()
    for nl, p, lo, hi in zip(batch["nls"], batch["ps"], b.offsets[:-1], b.offsets[1:]):
        og = O.build_graph(nl, p, nl["g0"][:, :2])
        want = O.apply_filter(nl, og, so, nl["g0"])
        U.check_filter(y[lo:hi], want, U.movable_rows(nl))


def test_graph_replays_match_direct_launch(batch):
    """Replays of the captured call, with other work and synchronisation in
    between, each equal the directly launched result."""
    b = batch["b"]
    spec = U.to_c_spec(A, BANK)
    other = U.to_c_spec(A, SPECS["sigma"])
    x = signal(batch, 4)
    b.set_config(4, 4, 4)
    eager = b.filter(spec, x, use_graph=False)
    torch.cuda.synchronize()
    out = torch.empty_like(x)
    for r in range(4):
        b.filter(spec, x, out=out)
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {r}"
        b.filter(other, x, use_graph=False)          # eager work between replays
        _ = (x * 2.0).sum()
        torch.cuda.synchronize()


def test_new_buffers_capture_again(batch):
    b = batch["b"]
    spec = U.to_c_spec(A, BANK)
    b.set_config(4, 2, 4)
    x1 = signal(batch, 4)
    x2 = (x1 + 3.0).contiguous()
    n0 = b.info()["n_captured"]
    y1 = b.filter(spec, x1).clone()
    y2 = b.filter(spec, x2).clone()
    assert b.info()["n_captured"] >= min(n0 + 1, 16)
    assert torch.equal(y1, b.filter(spec, x1, use_graph=False))
    assert torch.equal(y2, b.filter(spec, x2, use_graph=False))


def test_autotune_sets_a_valid_config(batch):
    b = batch["b"]
    spec = U.to_c_spec(A, BANK)
    lanes, ct, ms = b.autotune(spec, 4)
    print(f"tuned: lanes {lanes} tile {ct} {ms:.3f} ms")
    assert lanes in (1, 2, 4, 8, 16, 32, A.HOP_ROW_BLOCK) and ct in (1, 2, 4) and ms > 0
    assert b.get_config(4) == (lanes, ct)
    x = signal(batch, 4)
    A.filter_tune(lanes, -1)
    assert torch.equal(b.filter(spec, x), members_alone(batch, spec, x))


def test_single_member_batch_equals_graph(batch):
    nl, p = batch["nls"][1], batch["ps"][1]
    net = batch["nets"][1]
    x = torch.as_tensor(nl["g0"]).cuda()
    b1 = A.Batch([net], U.to_c_params(A, p), x)
    spec = U.to_c_spec(A, BANK)
    A.filter_tune(8, -1)
    b1.set_config(4, 8, 1)
    assert torch.equal(b1.filter(spec, x), batch["graphs"][1].filter(spec, x))
    b1.close()


def test_invalid_arguments(batch):
    b = batch["b"]
    with pytest.raises(A.AhrError):
        b.set_config(4, 3, 4)
    with pytest.raises(A.AhrError):
        b.set_config(4, 2, 8)
    with pytest.raises(A.AhrError):
        b.set_config(3, 2, 1)
    x = signal(batch, 4)
    with pytest.raises(A.AhrError):
        b.filter(U.to_c_spec(A, BANK), x, out=x)
