"""Caller-provided workspace (ahr_graph_workspace_size, ahr_graph_build with
ws, the netlist form of ahr_refine) through the C ABI: a graph whose device
memory is all carved from a torch-allocated workspace gives the same bits as
one on the library's pool, at small sizes and at the full mid-210k and
large-2.2M workloads, and never uses more than the size query returned;
workspaces below the bound are refused with AHR_ENOMEM and no handle."""
import ctypes

import numpy as np
import pytest
import torch

import gpu_common as U
import netlists as H
from oracle import ahr_oracle as O
from synth import netlist as N

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2511_10073_amd")

BANK = O.FilterSpec(ks=(2, 4, 8), alphas=(0.2, 0.3, 0.5))
CASES = [("tiny", N.TINY, dict(nbx=8, nby=8)),
         ("small-4col", N.small(7000, 4, ncols=4, big_frac=0.01), dict(nbx=16, nby=12, detection_ratio=0.2)),
         ("small-prune", N.small(7000, 4, ncols=4, big_frac=0.01), dict(nbx=16, nby=12, detection_ratio=0.2,
                                                                          prune_tau=0.2)),
         ("mid-210k", N.MID, dict(nbx=32, nby=32)),
         ("large-2.2M", N.LARGE, dict(nbx=32, nby=32))]


@pytest.mark.parametrize("name,cfg,kw", CASES, ids=[c[0] for c in CASES])
def test_workspace_graph_equals_pool_graph(name, cfg, kw):
    nl = N.generate(cfg)
    net = A.Netlist(nl)
    x = torch.as_tensor(nl["g0"]).cuda()
    C = x.shape[1]
    p = U.to_c_params(A, U.params32(O.HintParams(**kw)))
    spec = U.to_c_spec(A, U.spec32(BANK))
    need = A.workspace_size(net, p, C)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    g1 = A.Graph(net, p, x, ws=ws)
    g0 = A.Graph(net, p, x)
    try:
        r1 = g1.refine(spec, x, 3, 0.5)
        r0 = g0.refine(spec, x, 3, 0.5)
        f1 = g1.filter(spec, x)
        f0 = g0.filter(spec, x)
        torch.cuda.synchronize()
        inf = g1.info()
        assert inf["ws_bytes"] > 0 and 0 < inf["ws_peak"] <= inf["ws_bytes"] <= need
        assert g0.info()["ws_bytes"] == 0
        e1, e0 = g1.export(), g0.export()
    finally:
        g1.close()
        g0.close()
    assert torch.equal(r1, r0) and torch.equal(f1, f0)
    for k in ("net_row_ptr", "net_col", "net_q", "hint_row_ptr", "hint_col", "hint_val"):
        assert np.array_equal(e1[k], e0[k]), k
    print(f"[workspace] {name}: bound {need / 2**20:.1f} MiB, peak {inf['ws_peak'] / 2**20:.1f} MiB "
          f"({inf['ws_peak'] / need:.2f} of the bound)", flush=True)
    # Algorithm 1 end to end from the netlist, in a workspace
    r2 = A.refine(net, p, spec, x, 3, 0.5, ws=ws)
    torch.cuda.synchronize()
    assert torch.equal(r2, r0)


def test_workspace_below_the_bound_is_refused():
    nl = N.generate(N.small(3000, 5, ncols=2))
    net = A.Netlist(nl)
    x = torch.as_tensor(nl["g0"]).cuda()
    p = A.hint_params(nbx=8, nby=8)
    need = A.workspace_size(net, p, 2)
    ws = torch.empty(need - 4096, dtype=torch.uint8, device="cuda")
    lib = A.load()
    h = ctypes.c_void_p()
    rc = lib.ahr_graph_build(ctypes.byref(net.c), ctypes.byref(p), ctypes.c_void_p(x.data_ptr()), 2,
                             ctypes.c_void_p(ws.data_ptr()), ws.numel(), None, ctypes.byref(h))
    assert rc == A.ENOMEM and h.value is None
    assert b"workspace too small" in lib.ahr_last_error()
    out = torch.full_like(x, -7.0)
    spec = A.filter_spec((2, 4, 8), (0.2, 0.3, 0.5))
    with pytest.raises(A.AhrError) as e:
        A.refine(net, p, spec, x, 3, 0.5, out=out, ws=ws)
    assert e.value.code == A.ENOMEM
    torch.cuda.synchronize()
    assert torch.all(out == -7.0)


def test_clique_expansion_beyond_int32_is_unsupported():
    """One 50,000-pin net expanded as a clique (clique_max raised above its
    size) would have 50,000 x 49,999 > 2^31 entries: AHR_EUNSUPPORTED, no
    handle, and the library stays usable."""
    n = 50_000
    nl = H.make([list(range(n))], n, die=(-300, -300, 300, 300))
    net = A.Netlist(nl)
    x = torch.as_tensor(nl["g0"]).cuda()
    p = A.hint_params(nbx=8, nby=8, clique_max=100_000)
    with pytest.raises(A.AhrError) as e:
        A.Graph(net, p, x)
    assert e.value.code == A.EUNSUPPORTED
    assert "2^31" in str(e.value)
    g = A.Graph(net, A.hint_params(nbx=8, nby=8), x)       # as a star it is fine
    assert g.info()["first_star"] == n
    g.close()
