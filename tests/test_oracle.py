"""CPU pins of the FP64 oracle: each one fixes the oracle against something
other than itself -- brute force on tiny inputs, closed-form spectra, the
spectral definition of a graph filter, algebraic identities and invariants."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import netlists as H
from oracle import ahr_oracle as O
from synth import netlist as N

Q = 2 ** 32
NO_HINTS = O.HintParams(macro_hints=False, bin_hints=False)


def dense(g):
    return g.adjacency().toarray()


# ---------------------------------------------------------------- net model

def brute_netlist_q(nl, clique_max, expand=True):
    """Pure-Python accumulation of the clique/star integer weights."""
    n_inst = nl["n_inst"]
    flags = nl["node_flags"]
    node = [int(v) for v in nl["pin_node"]]
    nxt = n_inst
    if expand:
        for k, v in enumerate(node):
            if flags[v] & 1 and flags[v] & 2:
                node[k] = nxt
                nxt += 1
    acc = {}
    ptr = nl["net_ptr"]
    star = nxt
    for e in range(len(ptr) - 1):
        pins = node[ptr[e]:ptr[e + 1]]
        p = len(pins)
        if p < 2:
            continue
        if p <= clique_max:
            q = round(Q / (p - 1))            # exact for these small p (ties impossible)
            for a in pins:
                for b in pins:
                    if a != b:
                        acc[(a, b)] = acc.get((a, b), 0) + q
        else:
            qs = int(np.rint(Q * p / (p - 1)))
            for a in pins:
                acc[(a, star)] = acc.get((a, star), 0) + qs
                acc[(star, a)] = acc.get((star, a), 0) + qs
            star += 1
    return acc, star


@pytest.mark.parametrize("seed", [1, 2])
def test_netlist_csr_matches_brute_force(seed):
    nl = N.generate(N.small(300, seed, big_frac=0.02))
    g = O.build_graph(nl, NO_HINTS, nl["g0"][:, :2])
    acc, n_tot = brute_netlist_q(nl, 10)
    assert n_tot == g.n_tot
    got = {}
    for r in range(g.n_tot):
        cols = g.net_col[g.net_row_ptr[r]:g.net_row_ptr[r + 1]]
        assert np.all(np.diff(cols) > 0), "columns strictly ascending"
        for c, q in zip(cols, g.net_q[g.net_row_ptr[r]:g.net_row_ptr[r + 1]]):
            got[(r, int(c))] = int(q)
    assert got == acc


def test_clique_weights_single_net():
    # one 4-pin net: K_4 with weight 1/3 per pair, q = round(2^32/3)
    nl = H.make([[0, 1, 2, 3]], 4)
    g = O.build_graph(nl, NO_HINTS, nl["g0"])
    A = dense(g)
    assert np.allclose(A, (np.ones((4, 4)) - np.eye(4)) * round(Q / 3) / Q, rtol=0, atol=0)
    # normalised adjacency of K_p: eigenvalues 1 and -1/(p-1) (x p-1)
    d = A.sum(1)
    At = A / np.sqrt(np.outer(d, d))
    ev = np.sort(np.linalg.eigvalsh(At))
    assert np.allclose(ev, [-1 / 3] * 3 + [1], atol=1e-12)


def test_star_schur_complement_equals_clique():
    # a 12-pin net becomes a star; eliminating the hub gives the 12-clique
    # with w/(p-1) per pair (Laplacian Schur complement)
    p = 12
    nl = H.make([list(range(p))], p)
    g = O.build_graph(nl, NO_HINTS, nl["g0"])
    assert g.n_tot == p + 1 and g.star_net.tolist() == [0]
    A = dense(g)
    L = np.diag(A.sum(1)) - A
    Lss = L[:p, :p] - np.outer(L[:p, p], L[p, :p]) / L[p, p]
    Kc = (np.ones((p, p)) - np.eye(p)) / (p - 1)
    assert np.allclose(Lss, np.diag(Kc.sum(1)) - Kc, atol=1e-9)
    # star K_{1,p}: normalised adjacency eigenvalues +-1 and 0 (x p-1)
    d = A.sum(1)
    ev = np.sort(np.linalg.eigvalsh(A / np.sqrt(np.outer(d, d))))
    assert np.allclose(ev, [-1] + [0] * (p - 1) + [1], atol=1e-12)


def test_quadratic_form_is_wirelength():
    # Section IV: the quadratic wirelength of the clique model equals g^T L g
    nl = N.generate(N.small(200, 5))
    g = O.build_graph(nl, NO_HINTS, nl["g0"][:, :2])
    A = dense(g)
    x = np.random.default_rng(3).normal(size=g.n_tot)
    L = np.diag(A.sum(1)) - A
    iu = np.triu_indices(g.n_tot, 1)
    s = np.sum(A[iu] * (x[iu[0]] - x[iu[1]]) ** 2)
    assert math.isclose(x @ L @ x, s, rel_tol=1e-10)


def test_macro_pin_expansion():
    # node 2 is a fixed macro with 3 pins on 3 nets; node 3 a movable macro
    flags = [0, 0, H.FIXED | H.MACRO, H.MACRO]
    nets = [[0, 2], [1, 2], [2, 3, 0]]
    off = np.array([[0, 0], [1, 0], [0, 0], [0, 2], [0, 0], [0, 0], [0, 0]], np.float32)
    nl = H.make(nets, 4, flags=flags, offsets=off)
    g = O.build_graph(nl, NO_HINTS, nl["g0"])
    assert g.first_mpin == 4 and g.first_star == 7
    assert g.mpin_owner.tolist() == [2, 2, 2] and g.mpin_pin.tolist() == [1, 3, 4]
    A = dense(g)
    assert np.all(A[2] == 0) and np.all(A[:, 2] == 0)          # macro instance isolated
    assert A[0, 4] > 0 and A[1, 5] > 0 and A[3, 6] > 0 and A[0, 6] > 0
    X = O.expand_signal(nl, g, nl["g0"])
    assert np.allclose(X[4], nl["g0"][2] + [1, 0])
    assert np.allclose(X[5], nl["g0"][2] + [0, 2])
    assert g.pinned[4:7].all() and g.pinned[2] and not g.pinned[3]


# ---------------------------------------------------------------- operator

def ring_graph(n):
    nl = H.ring(n)
    return nl, O.build_graph(nl, NO_HINTS, nl["g0"])


def test_cycle_spectrum_closed_form():
    n = 17
    _, g = ring_graph(n)
    L, T, d, s, lam = O.operator(g)
    ev = np.sort(np.linalg.eigvalsh(L.toarray()))
    ref = np.sort(1 - np.cos(2 * np.pi * np.arange(n) / n))
    assert np.allclose(ev, ref, atol=1e-12)
    assert math.isclose(lam, 2.0, rel_tol=1e-15)     # Gershgorin: 1 + 2 * 1/2


def test_signed_cycle_spectrum_closed_form():
    # replace one ring edge by a negative one: eigenvalues 1 - cos((2k+1) pi / n)
    n = 13
    nl = H.make([[i, i + 1] for i in range(n - 1)], n)
    g = O.build_graph(nl, NO_HINTS, nl["g0"])
    g.hint_row_ptr = np.zeros(n + 1, np.int64)
    g.hint_row_ptr[1:n] = 1
    g.hint_row_ptr[n] = 2
    g.hint_row_ptr[0] = 0
    # rows 0 and n-1 carry the negative edge (0, n-1)
    cnt = np.zeros(n, np.int64)
    cnt[0] = cnt[n - 1] = 1
    g.hint_row_ptr = np.concatenate([[0], np.cumsum(cnt)])
    g.hint_col = np.array([n - 1, 0])
    g.hint_val = np.array([-1.0, -1.0])
    L, _, _, _, _ = O.operator(g)
    ev = np.sort(np.linalg.eigvalsh(L.toarray()))
    ref = np.sort(1 - np.cos((2 * np.arange(n) + 1) * np.pi / n))
    assert np.allclose(ev, ref, atol=1e-12)


def tiny_hint_graph(seed=11, **kw):
    nl = N.generate(N.small(400, seed, movable_macros=kw.pop("movable", False)))
    kw.setdefault("nbx", 8)
    kw.setdefault("nby", 8)
    p = O.HintParams(**kw)
    return nl, O.build_graph(nl, p, nl["g0"][:, :2])


def test_signed_quadratic_form_and_psd():
    nl, g = tiny_hint_graph()
    A = dense(g)
    assert np.array_equal(A, A.T)
    assert (A < 0).sum() > 0 and (A > 0).sum() > 0
    L, T, d, s, lam = O.operator(g)
    x = np.random.default_rng(2).normal(size=g.n_tot)
    iu = np.triu_indices(g.n_tot, 1)
    a = A[iu]
    y = s * x
    rhs = np.sum(np.abs(a) * (y[iu[0]] - np.sign(a) * y[iu[1]]) ** 2)
    assert math.isclose(x @ (L @ x), rhs, rel_tol=1e-9)
    ev = np.linalg.eigvalsh(L.toarray())
    assert ev.min() >= -1e-12 and ev.max() <= 2 + 1e-12 and ev.max() <= lam + 1e-12


@pytest.mark.parametrize("sigma", [0.0, 0.5])
def test_filter_equals_spectral_definition(sigma):
    # Section II-A eq. "filter": H = U h(Lambda) U^T with h(l) = sum a (1 - l/lup)^k
    nl, g = tiny_hint_graph()
    spec = O.FilterSpec(ks=(2, 4, 8), alphas=(0.2, 0.3, 0.5), sigma=sigma)
    L, T, d, s, lam = O.operator(g, sigma=sigma)
    out, lam2 = O.apply_filter(nl, g, spec, nl["g0"], return_full=True, pin=False)
    assert lam == lam2
    ev, U = np.linalg.eigh(L.toarray())
    h = sum(a * (1 - ev / lam) ** k for k, a in zip(spec.ks, spec.alphas))
    X = O.expand_signal(nl, g, nl["g0"])
    ref = U @ (h[:, None] * (U.T @ X))
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(X)) * 10


def test_unsigned_degree_eigenvector():
    # without negative edges D^{1/2} 1 is the eigenvalue-1 eigenvector of T
    nl = N.generate(N.small(500, 4))
    g = O.build_graph(nl, NO_HINTS, nl["g0"][:, :2])
    spec = O.FilterSpec(ks=(2, 4, 8), alphas=(0.2, 0.3, 0.5))
    L, T, d, s, lam = O.operator(g)
    v = np.sqrt(d)
    assert np.allclose(T @ v, v, atol=1e-12 * v.max())
    # the filter is linear on the expanded signal: feed v through the chain
    Y, out = v.copy(), np.zeros_like(v)
    for j in range(1, 9):
        Y = T @ Y
        out += {2: 0.2, 4: 0.3, 8: 0.5}.get(j, 0) * Y
    assert np.allclose(out, v, atol=1e-11 * v.max())


def test_special_cases_identity_and_textbook_adjacency():
    nl, g = tiny_hint_graph()
    G = nl["g0"]
    X = O.expand_signal(nl, g, G)
    out0, _ = O.apply_filter(nl, g, O.FilterSpec(ks=(0,), alphas=(1.0,)), G, return_full=True, pin=False)
    assert np.array_equal(out0, X)
    # K=1 with lambda_up fixed to 1 is one product with D^{-1/2} A D^{-1/2}
    out1, _ = O.apply_filter(nl, g, O.FilterSpec(ks=(1,), alphas=(1.0,), lambda_mode="fixed",
                                                 lambda_fixed=1.0), G, return_full=True, pin=False)
    A = dense(g)
    d = np.abs(A).sum(1)
    with np.errstate(divide="ignore"):
        r = np.where(d > 0, 1 / np.sqrt(d), 0)
    ref = (r[:, None] * A * r[None, :]) @ X + (d == 0)[:, None] * X
    assert np.allclose(out1, ref, atol=1e-12 * np.abs(X).max())


def test_pinned_rows_equal_input():
    nl, g = tiny_hint_graph()
    spec = O.FilterSpec(ks=(2, 4, 8), alphas=(0.2, 0.3, 0.5))
    out, _ = O.apply_filter(nl, g, spec, nl["g0"], return_full=True)
    X = O.expand_signal(nl, g, nl["g0"])
    assert np.array_equal(out[g.pinned], X[g.pinned])
    assert not np.allclose(out[~g.pinned], X[~g.pinned])


# ---------------------------------------------------------------- hints

def test_bin_membership_and_window():
    nl, g = tiny_hint_graph()
    gr = g.grid
    pos = nl["g0"][:, :2]
    fixed, macro, std = O.node_kinds(nl)
    cells = np.flatnonzero(std)
    bx, by = O.cell_bin(gr, pos[cells, 0], pos[cells, 1])
    # geometric containment (interior cells; clamped at the die border)
    x = pos[cells, 0].astype(np.float64)
    lo = gr.xl + bx * gr.bw
    inside = (x >= gr.xl) & (x < gr.xl + gr.nbx * gr.bw)
    assert np.all((x[inside] >= lo[inside] - 1e-4) & (x[inside] <= lo[inside] + gr.bw + 1e-4))
    # every hint cell has exactly the clipped 3x3 (8x8 grid -> n=1 -> 1x1) window
    hx = O.window_half(0.1, 8)
    assert hx == 0 and O.window_half(0.1, 32) == 1 and O.window_half(0.1, 10) == 0
    A = dense(g)
    hint_cells = cells[g.qdeg[cells] > 0]
    nb = A[hint_cells][:, g.first_bvirt:]
    assert np.all((nb != 0).sum(1) <= 1)


def test_density_conserves_area_and_phi_sign():
    nl, g = tiny_hint_graph()
    gr = g.grid
    fixed, macro, std = O.node_kinds(nl)
    size = nl["node_size"].astype(np.float64)
    pos = nl["g0"][:, :2].astype(np.float64)
    total = g.density.sum() * gr.bw * gr.bh
    cell_area = (size[std, 0] * size[std, 1]).sum()
    d = nl["die"].astype(np.float64)
    mac = 0.0
    for m in np.flatnonzero(macro):
        ox = max(0.0, min(pos[m, 0] + size[m, 0] / 2, d[2]) - max(pos[m, 0] - size[m, 0] / 2, d[0]))
        oy = max(0.0, min(pos[m, 1] + size[m, 1] / 2, d[3]) - max(pos[m, 1] - size[m, 1] / 2, d[1]))
        mac += ox * oy
    assert math.isclose(total, cell_area + mac, rel_tol=1e-12)
    # phi = tanh(mu (D - C) / 2), sign follows overfull / underfull
    assert np.allclose(g.phi, np.tanh(4.0 * (g.density - 1.0) / 2), atol=1e-14)
    assert np.all(np.sign(g.phi) == np.sign(g.density - 1.0))


def brute_density(nl, nbx, nby, pos):
    """Per-bin density by loops: each movable std cell's area goes to the bin
    holding its centre (float32 decision, clamped), each macro's footprint is
    clipped against every bin rectangle."""
    d = [float(v) for v in nl["die"]]
    bw, bh = (d[2] - d[0]) / nbx, (d[3] - d[1]) / nby
    bw32 = np.float32(np.float32(nl["die"][2] - nl["die"][0]) / np.float32(nbx))
    bh32 = np.float32(np.float32(nl["die"][3] - nl["die"][1]) / np.float32(nby))
    area = [0.0] * (nbx * nby)
    for i in range(nl["n_inst"]):
        f = int(nl["node_flags"][i])
        w, h = float(nl["node_size"][i, 0]), float(nl["node_size"][i, 1])
        x, y = np.float32(pos[i, 0]), np.float32(pos[i, 1])
        if f == 0:
            bx = min(max(int(math.floor(np.float32((x - nl["die"][0]) / bw32))), 0), nbx - 1)
            by = min(max(int(math.floor(np.float32((y - nl["die"][1]) / bh32))), 0), nby - 1)
            area[by * nbx + bx] += w * h
        elif f & 2:
            for by in range(nby):
                for bx in range(nbx):
                    x0, x1 = d[0] + bx * bw, d[0] + (bx + 1) * bw
                    y0, y1 = d[1] + by * bh, d[1] + (by + 1) * bh
                    ox = min(float(x) + w / 2, x1) - max(float(x) - w / 2, x0)
                    oy = min(float(y) + h / 2, y1) - max(float(y) - h / 2, y0)
                    if ox > 0 and oy > 0:
                        area[by * nbx + bx] += ox * oy
    return [a / (bw * bh) for a in area]


def test_brute_density_matches_oracle():
    nl, g = tiny_hint_graph(movable=True, nbx=10, nby=7)
    ref = brute_density(nl, 10, 7, nl["g0"][:, :2])
    assert np.allclose(g.density, ref, rtol=1e-12, atol=1e-15)


def test_hint_edges_brute_force():
    nl, g = tiny_hint_graph(movable=True, nbx=10, nby=10, detection_ratio=0.3)
    gr = g.grid
    pos = nl["g0"][:, :2]
    fixed, macro, std = O.node_kinds(nl)
    size = nl["node_size"]
    A = dense(g)
    hx = O.window_half(0.3, 10)
    assert hx == 1
    # phi_b and baseWeight from their definitions, not from the oracle's graph
    dens = brute_density(nl, 10, 10, pos)
    phis = [2.0 / (1.0 + math.exp(-4.0 * (D - 1.0))) - 1.0 for D in dens]
    acc, _ = brute_netlist_q(nl, 10)
    qsum, cnt = {}, {}
    for (r, c), q in acc.items():
        qsum[r] = qsum.get(r, 0) + q
        cnt[r] = cnt.get(r, 0) + 1
    checked = 0
    for i in np.flatnonzero(std):
        if i not in cnt:
            assert g.qdeg[i] == 0
            assert np.all(A[i, g.first_mvirt:] == 0)
            continue
        bwi = qsum[i] / Q / cnt[i]
        x32, y32 = np.float32(pos[i, 0]), np.float32(pos[i, 1])
        bxi = min(max(int(math.floor(float(np.float32((x32 - gr.xl32) / gr.bw32)))), 0), gr.nbx - 1)
        byi = min(max(int(math.floor(float(np.float32((y32 - gr.yl32) / gr.bh32)))), 0), gr.nby - 1)
        for b in range(gr.nbx * gr.nby):
            bx, by = b % gr.nbx, b // gr.nbx
            want = abs(bx - bxi) <= hx and abs(by - byi) <= hx
            v = A[i, g.first_bvirt + b]
            if not want:
                assert v == 0
                continue
            cx = gr.xl + (bx + 0.5) * gr.bw
            cy = gr.yl + (by + 0.5) * gr.bh
            mr = max(abs(float(x32) - cx) / (gr.bw / 2), abs(float(y32) - cy) / (gr.bh / 2))
            ref = -math.exp(-mr) * phis[b] * bwi
            assert math.isclose(v, ref, rel_tol=1e-12, abs_tol=1e-300)
            checked += 1
        for k, m in enumerate(g.macro_ids):
            mx, my = np.float32(pos[m, 0]), np.float32(pos[m, 1])
            ins = (abs(x32 - mx) <= size[m, 0] / np.float32(2)) and (abs(y32 - my) <= size[m, 1] / np.float32(2))
            v = A[i, g.first_mvirt + k]
            if ins:
                mr = max(abs(float(x32) - float(mx)) / (float(size[m, 0]) / 2),
                         abs(float(y32) - float(my)) / (float(size[m, 1]) / 2))
                assert mr <= 1.0 + 1e-6
                assert math.isclose(v, -math.exp(-mr) * bwi, rel_tol=1e-12)
            else:
                assert v == 0
    assert checked > 1000


# ---------------------------------------------------------------- Algorithm 1, HPWL

def test_refine_special_cases():
    nl = N.generate(N.small(300, 8))
    p = O.HintParams(nbx=8, nby=8)
    spec = O.FilterSpec(ks=(4,), alphas=(1.0,))
    G0 = nl["g0"]
    assert np.array_equal(O.refine(nl, p, spec, G0, 0, 0.5), G0.astype(np.float64))
    assert np.array_equal(O.refine(nl, p, spec, G0, 3, 0.0), G0.astype(np.float64))
    g = O.build_graph(nl, p, G0[:, :2])
    one = O.refine(nl, p, spec, G0, 1, 1.0)
    assert np.allclose(one, O.apply_filter(nl, g, spec, G0), rtol=0, atol=1e-12)
    three = O.refine(nl, p, spec, G0, 3, 0.5)
    fixed = (nl["node_flags"] & 1) != 0
    assert np.array_equal(three[fixed], G0[fixed].astype(np.float64))


def test_hpwl_brute_force_and_closed_form():
    nl = H.make([[0, 1]], 2, pos=[[0, 0], [3, 4]])
    tot, _ = O.hpwl(nl, nl["g0"])
    assert tot[0] == 7.0
    nl = N.generate(N.small(300, 9, ncols=4))
    tot, per = O.hpwl(nl, nl["g0"])
    ptr, node, off, G = nl["net_ptr"], nl["pin_node"], nl["pin_off"], nl["g0"].astype(np.float64)
    for c in range(2):
        s = 0.0
        for e in range(len(ptr) - 1):
            xs = [G[node[k], 2 * c] + float(off[k, 0]) for k in range(ptr[e], ptr[e + 1])]
            ys = [G[node[k], 2 * c + 1] + float(off[k, 1]) for k in range(ptr[e], ptr[e + 1])]
            s += (max(xs) - min(xs)) + (max(ys) - min(ys))
        assert math.isclose(tot[c], s, rel_tol=1e-12)
