"""CPU pins of the GiFt oracle (Section IV eqs. "GiFt" and "GiFt filter"):
the closed-form spectrum of the augmented operator on a cycle (applied
through the discrete Fourier transform), the D_sigma^1/2 1 eigenvector,
dense eigendecompositions on a weighted netlist with star nodes, the large
sigma limit and the pinning of fixed rows."""
import numpy as np
import pytest

import netlists as H
from oracle import ahr_oracle as O
from synth import netlist as N

GIFT_GRAPH = O.HintParams(expand_macro_pins=False, macro_hints=False, bin_hints=False)


def test_cycle_spectrum_through_the_fourier_basis():
    """On the unit cycle C_n every degree is 2, so Atilde_sigma =
    (A + sigma I)/(2 + sigma), whose eigenvalue at frequency 2 pi j / n is
    (2 cos(2 pi j / n) + sigma)/(2 + sigma); the bank multiplies each Fourier
    coefficient by sum_b alpha_b of its k_b-th power."""
    n = 64
    nl = H.ring(n)
    g = O.build_graph(nl, GIFT_GRAPH, nl["g0"])
    bank = O.GiftBank()
    x = np.random.default_rng(4).normal(size=(n, 2))
    out = O.gift(nl, g, bank, x, pin=False)
    th = 2 * np.pi * np.arange(n) / n
    h = sum(a * ((2 * np.cos(th) + s) / (2 + s)) ** k for k, s, a in zip(bank.ks, bank.sigmas, bank.alphas))
    ref = np.real(np.fft.ifft(h[:, None] * np.fft.fft(x, axis=0), axis=0))
    assert np.allclose(out, ref, rtol=0, atol=1e-13)


def test_degree_vector_is_an_eigenvector():
    # Atilde_sigma D_sigma^1/2 1 = D_sigma^-1/2 (d + sigma) = D_sigma^1/2 1 for every sigma
    nl = N.generate(N.small(400, 22, big_frac=0.02))
    g = O.build_graph(nl, GIFT_GRAPH, nl["g0"][:, :2])
    A = g.adjacency()
    d = np.asarray(A.sum(axis=1)).ravel()
    for s in (2.0, 4.0):
        v = np.sqrt(d + s)
        assert np.allclose(O.gift_operator(g, s) @ v, v, rtol=1e-12, atol=0)
    bank = O.GiftBank()
    # the bank on the expanded signal: feed v for one sigma through its bands
    vs = np.sqrt(d + 4.0)
    At = O.gift_operator(g, 4.0)
    out = 0.3 * (At @ (At @ vs)) + 0.5 * (At @ (At @ (At @ (At @ vs))))
    assert np.allclose(out, 0.8 * vs, rtol=1e-12)


@pytest.mark.parametrize("seed", [23, 24])
def test_bank_equals_dense_eigendecompositions(seed):
    """H X = sum_b alpha_b U_b diag(mu_b^k_b) U_b^T X with (mu_b, U_b) the
    eigenpairs of the dense symmetric Atilde_{sigma_b} (weighted cliques and
    stars, float net weights)."""
    nl = N.generate(N.small(250, seed, big_frac=0.05))
    nl["net_w"] = np.random.default_rng(seed).uniform(0.5, 2.0, nl["net_ptr"].size - 1).astype(np.float32)
    g = O.build_graph(nl, GIFT_GRAPH, nl["g0"][:, :2])
    bank = O.GiftBank(ks=(2, 2, 4), sigmas=(2.0, 4.0, 4.0), alphas=(0.25, 0.25, 0.5))
    X = O.expand_signal(nl, g, nl["g0"])
    out = O.gift(nl, g, bank, nl["g0"], pin=False, return_full=True)
    A = g.adjacency().toarray()
    d = A.sum(axis=1)
    ref = np.zeros_like(X)
    for k, s, a in zip(bank.ks, bank.sigmas, bank.alphas):
        r = 1.0 / np.sqrt(d + s)
        At = r[:, None] * (A + s * np.eye(A.shape[0])) * r[None, :]
        mu, U = np.linalg.eigh(At)
        ref += a * (U @ ((mu ** k)[:, None] * (U.T @ X)))
    assert np.allclose(out, ref, rtol=0, atol=1e-11 * np.abs(X).max())


def test_large_sigma_is_the_identity():
    nl = N.generate(N.small(200, 25))
    g = O.build_graph(nl, GIFT_GRAPH, nl["g0"][:, :2])
    bank = O.GiftBank(sigmas=(1e12, 1e12, 1e12))
    out = O.gift(nl, g, bank, nl["g0"], pin=False)
    assert np.allclose(out, nl["g0"], rtol=1e-9, atol=1e-9)


def test_fixed_rows_reset_and_star_values():
    nl = N.generate(N.small(300, 26, big_frac=0.03))
    g = O.build_graph(nl, GIFT_GRAPH, nl["g0"][:, :2])
    assert g.star_net.size > 0 and g.first_mpin == g.first_star      # stars, no macro pin nodes
    out = O.gift(nl, g, O.GiftBank(), nl["g0"])
    fixed = (nl["node_flags"] & 1) != 0
    assert np.array_equal(out[fixed], nl["g0"][fixed].astype(np.float64))
    assert not np.allclose(out[~fixed], nl["g0"][~fixed])
