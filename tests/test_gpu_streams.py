"""Graph lifetimes and streams, through the C ABI.

A graph whose work all went to one stream is freed without waiting for the
device: its memory goes back to the allocator in that stream's order.
Graphs built right after it -- on the same stream and on another one --
reuse that memory while the first graph's kernels may still be running,
and must give the same bits as a graph built and run alone.  A graph used
on two streams is freed with a device wait, and the same holds."""
import numpy as np
import pytest
import torch

import gpu_common as U
from oracle import ahr_oracle as O
from synth import netlist as N

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2511_10073_amd")


def setup():
    nl = N.generate(N.TINY)
    net = A.Netlist(nl)
    x = torch.as_tensor(nl["g0"]).cuda()
    p = U.to_c_params(A, U.params32(O.HintParams(nbx=8, nby=8)))
    spec = U.to_c_spec(A, U.spec32(O.FilterSpec(ks=(2, 4, 8), alphas=(0.2, 0.3, 0.5))))
    torch.cuda.synchronize()
    return net, x, p, spec


def refine_alone(net, x, p, spec):
    gr = A.Graph(net, p, x)
    out = gr.refine(spec, x, 2, 0.5)
    torch.cuda.synchronize()
    gr.close()
    return out


def test_free_without_wait_then_reuse_on_same_and_other_stream():
    net, x, p, spec = setup()
    ref = refine_alone(net, x, p, spec)
    side = torch.cuda.Stream()
    main = torch.cuda.current_stream()
    side.wait_stream(main)
    outs = []
    for _ in range(3):
        with torch.cuda.stream(side):
            g1 = A.Graph(net, p, x, stream=side)
            o1 = g1.refine(spec, x, 2, 0.5, stream=side)
            g1.close()                                  # no device wait
            g2 = A.Graph(net, p, x, stream=side)        # same stream: reuses g1's blocks in order
            o2 = g2.refine(spec, x, 2, 0.5, stream=side)
            g2.close()
        g3 = A.Graph(net, p, x, stream=main)            # other stream: reuses behind the free events
        o3 = g3.refine(spec, x, 2, 0.5, stream=main)
        g3.close()
        outs += [o1, o2, o3]
    torch.cuda.synchronize()
    for o in outs:
        assert torch.equal(o, ref)


def test_graph_on_two_streams_freed_with_wait():
    net, x, p, spec = setup()
    ref = refine_alone(net, x, p, spec)
    side = torch.cuda.Stream()
    main = torch.cuda.current_stream()
    side.wait_stream(main)
    gr = A.Graph(net, p, x, stream=main)
    o1 = gr.refine(spec, x, 2, 0.5, stream=main)
    side.wait_stream(main)
    with torch.cuda.stream(side):
        o2 = gr.refine(spec, x, 2, 0.5, stream=side)
    main.wait_stream(side)
    gr.close()                                          # two streams: waits for the device
    g2 = A.Graph(net, p, x, stream=main)
    o3 = g2.refine(spec, x, 2, 0.5, stream=main)
    g2.close()
    torch.cuda.synchronize()
    for o in (o1, o2, o3):
        assert torch.equal(o, ref)


def test_graph_on_two_streams_closed_without_join():
    """close() of a graph whose last work went to a non-blocking stream that
    was never joined back: the destructor waits for the device before the
    memory can be taken by a graph on a third stream."""
    net, x, p, spec = setup()
    ref = refine_alone(net, x, p, spec)
    side, third = torch.cuda.Stream(), torch.cuda.Stream()
    main = torch.cuda.current_stream()
    side.wait_stream(main)
    third.wait_stream(main)
    outs = []
    for _ in range(3):
        gr = A.Graph(net, p, x, stream=main)
        outs.append(gr.refine(spec, x, 2, 0.5, stream=main))
        side.wait_stream(main)
        outs.append(gr.refine(spec, x, 2, 0.5, stream=side))
        gr.close()                                      # side not joined: the close waits for the device
        g2 = A.Graph(net, p, x, stream=third)
        outs.append(g2.refine(spec, x, 2, 0.5, stream=third))
        g2.close()
    torch.cuda.synchronize()
    for o in outs:
        assert torch.equal(o, ref)


def test_hpwl_calls_overlap_on_two_streams():
    """ahr_hpwl's partial sums are per call: two streams computing HPWL of
    different placements at the same time get what each gets alone."""
    net, x, p, spec = setup()
    y = x.clone()
    y[:, 0] *= 0.5
    ref_x = A.hpwl(net, x).clone()
    ref_y = A.hpwl(net, y).clone()
    torch.cuda.synchronize()
    assert not torch.equal(ref_x, ref_y)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    ox, oy = [], []
    for _ in range(50):
        ox.append(A.hpwl(net, x, stream=s1))
        oy.append(A.hpwl(net, y, stream=s2))
    torch.cuda.synchronize()
    for a, b in zip(ox, oy):
        assert torch.equal(a, ref_x) and torch.equal(b, ref_y)
