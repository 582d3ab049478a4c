"""CPU pins of the learned-surrogate oracle: the backward pass against
central finite differences, the bfloat16 rounding against torch's own
conversion and hand cases, and the features against their definitions."""
import numpy as np
import pytest
import torch

from oracle import ahr_oracle as O
from oracle import mlp_oracle as M
from synth import netlist as N


def test_bf16_rounding_matches_torch_and_ties_to_even():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 10000), rng.normal(0, 1e6, 1000), [0.0, -0.0, 1.0, -2.5]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(x), ref)
    # 1 + 2^-8 is halfway between bfloat16 1 and 1 + 2^-7: ties to even -> 1
    assert M.bf16(np.float32(1 + 2.0 ** -8)) == 1.0
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: ties to even -> 1 + 2^-6
    assert M.bf16(np.float32(1 + 3 * 2.0 ** -8)) == 1 + 2.0 ** -6
    assert M.bf16(np.float32(1 + 2.0 ** -8 + 2.0 ** -20)) == 1 + 2.0 ** -7


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    p = M.init_params(3).astype(np.float64)
    p[M.OFFSETS["b1"][0]:M.OFFSETS["b1"][0] + 64] = rng.normal(0, 0.1, 64)
    F = rng.normal(0, 1, (40, M.NFEAT))
    r = rng.normal(0, 1, 40)
    loss, g = M.loss_grad(p, F, r, rounding=False)
    idx = np.concatenate([rng.choice(M.NPARAM, 60, replace=False),
                          [M.OFFSETS["b3"][0], M.OFFSETS["w3"][0], M.OFFSETS["W1"][0]]])
    eps = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += eps
        pm[k] -= eps
        fd = (M.loss_grad(pp, F, r, rounding=False)[0] - M.loss_grad(pm, F, r, rounding=False)[0]) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-8, (k, fd, g[k])
    # padding features never receive gradient through zero inputs
    W1 = g[:M.HIDDEN * M.FEAT_PAD].reshape(M.HIDDEN, M.FEAT_PAD)
    assert np.all(W1[:, M.NFEAT:] == 0)


def test_forward_closed_forms():
    F = np.random.default_rng(2).normal(0, 1, (10, M.NFEAT))
    zero = np.zeros(M.NPARAM)
    zero[M.OFFSETS["b3"][0]] = 0.75
    o, _ = M.forward(zero, F)
    assert np.all(o == 0.75)
    # relu(f0) through one hidden unit: W1[0,0] = 1, W2[0,0] = 1, w3[0] = 2  ->  o = 2 relu(bf16(f0))
    p = np.zeros(M.NPARAM)
    W1o, W2o, w3o = M.OFFSETS["W1"][0], M.OFFSETS["W2"][0], M.OFFSETS["w3"][0]
    p[W1o] = 1.0
    p[W2o] = 1.0
    p[w3o] = 2.0
    o, _ = M.forward(p, F)
    assert np.allclose(o, 2 * np.maximum(M.bf16(F[:, 0].astype(np.float32)), 0), rtol=0, atol=0)


def test_features_follow_their_definitions():
    nl = N.generate(N.small(400, 21, ncols=4))
    g = O.build_graph(nl, O.HintParams(nbx=8, nby=8), nl["g0"][:, :2])
    F, (h0, h1, h2, h3), (m, s, r) = M.features(nl, g, nl["g0"])
    # h_0 is the input; h_j equal single-band filters without pinning
    assert np.array_equal(h0, np.asarray(nl["g0"], np.float64))
    for j, h in ((1, h1), (2, h2), (3, h3)):
        ref, _ = O.apply_filter(nl, g, O.FilterSpec(ks=(j,), alphas=(1.0,)), nl["g0"], return_full=True, pin=False)
        assert np.allclose(h, ref[:g.n_inst], rtol=0, atol=1e-12 * np.abs(ref).max())
    mov = (nl["node_flags"] & 1) == 0
    # feature 3 is standardised h_3; feature 0 has unit root mean square (r_c's definition)
    assert np.allclose(F[mov, :, 3].mean(axis=0), 0, atol=1e-9)
    assert np.allclose(F[mov, :, 3].std(axis=0), 1, atol=1e-9)
    assert np.allclose(np.sqrt(np.mean(F[mov, :, 0] ** 2, axis=0)), 1, atol=1e-12)
    # features 1 and 2 share feature 0's scale: their ratios to it are the hops' own
    i = np.flatnonzero(mov)[:20]
    for k, h in ((1, h1), (2, h2)):
        assert np.allclose(F[i, :, k] * r, h[i] - h3[i], rtol=1e-12, atol=1e-9 * np.abs(h3).max())
    assert np.allclose(F[:, :, 6], np.log(s / r)[None, :])
    A = g.adjacency().toarray()
    d = np.abs(A).sum(1)
    hint = A[:, g.first_mvirt:].sum(1)
    i = np.flatnonzero(mov & (d[:g.n_inst] > 0))[:50]
    assert np.allclose(F[i, 0, 5], hint[i] / d[i])
    assert np.allclose(F[i, 0, 4], np.log1p(d[i]))


def test_zero_network_with_the_bank_coefficients_is_the_filter():
    """A bank of order at most 3 lies in the span of h_0..h_3: with a zero
    network and beta set to the bank's weights, the surrogate is the plain
    filter of Section V (fixed rows pinned as there)."""
    nl = N.generate(N.small(500, 23, ncols=4))
    g = O.build_graph(nl, O.HintParams(nbx=8, nby=8), nl["g0"][:, :2])
    spec = O.FilterSpec(ks=(0, 1, 3), alphas=(0.1, 0.25, 0.65))
    ref = O.apply_filter(nl, g, spec, nl["g0"])
    zero = np.zeros(M.NPARAM)
    y = M.learned_filter(nl, g, zero, (0.1, 0.25, 0.0, 0.65), nl["g0"])
    assert np.allclose(y, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    # the network's output enters scaled by r_c
    b3 = np.zeros(M.NPARAM)
    b3[M.OFFSETS["b3"][0]] = 0.5
    F, h, (m, s, r) = M.features(nl, g, nl["g0"])
    y2 = M.learned_filter(nl, g, b3, (0.1, 0.25, 0.0, 0.65), nl["g0"])
    mov = (nl["node_flags"] & 1) == 0
    assert np.allclose(y2[mov] - y[mov], 0.5 * r[None, :], rtol=1e-12)


def test_column_stats_fall_back_to_one():
    h0 = np.array([[1.0, 2.0], [3.0, 2.0]])
    h3 = np.array([[5.0, 2.0], [5.0, 2.0]])
    m, s, r = M.column_stats(h0, h3, np.array([True, True]))
    assert np.array_equal(m, [5.0, 2.0])
    assert np.array_equal(s, [1.0, 1.0])          # h_3 constant
    assert np.allclose(r, [np.sqrt(10.0), 1.0])   # RMS of (-4, -2); zero in column 1
