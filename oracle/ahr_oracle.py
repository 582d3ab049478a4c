"""FP64 CPU oracle of the signed netlist graph filter (area-hint refinement).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP library: it reads the
same seeded input arrays (from ``synth``) and nothing else.

Every function cites the passage of the paper (arXiv 2511.10073) it follows.
Where the paper is silent the reading adopted is named in the docstring
(readings R1..R20 are listed in the design notes).  Arithmetic is float64
except the structural decisions (which bin a cell is in, whether a cell lies
inside a macro footprint, the detection-window size), which are taken in IEEE
float32 so that the GPU, which takes them in float32 too, reaches the same
integers.

The method, in the paper's order:
  * Section IV: a placement instance is a graph whose objects are nodes and
    whose nets are edges; the quadratic wirelength is the graph's smoothness
    (eq. "Wirelength objective").
  * Section V, "Macro pin expansion": a fixed macro is split into fixed nodes
    at its pin sites.
  * Section V, "Macro virtual node": one virtual node per macro, negative
    edges -exp(-maxRatio) * baseWeight to movable cells in its footprint.
  * Section V, "Bin virtual node": one virtual node per bin, signed edges
    -exp(-maxRatio) * phi_b * baseWeight, phi_b = 2 sigmoid(mu (D_b - C)) - 1,
    to movable cells in an n_x x n_y window.
  * Section V, eq. "refine-filter": H_r = ((lambda_up I - L_hint)/lambda_up)^k,
    lambda_up from the Gershgorin circle theorem.
  * Section V, Algorithm 1: T_hint rounds of build / filter / relax.
  * HPWL, the paper's wirelength score (Section VII, evaluation metrics).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

FLAG_FIXED = 1
FLAG_MACRO = 2

Q_SCALE = 2.0 ** 32        # netlist weights are kept as integers in units of 2^-32


@dataclasses.dataclass
class HintParams:
    """Area-hint parameters (Section V; Table "Parameter space", refinement block)."""
    nbx: int = 8
    nby: int = 8
    detection_ratio: float = 0.1   # window n = max(1, floor(ratio * numBin))
    bin_capacity: float = 1.0      # C, the target per-bin density
    mu: float = 4.0                # slope of the logistic map (mu > 0)
    clique_max: int = 10           # nets with p <= clique_max become cliques, else stars
    expand_macro_pins: bool = True
    macro_hints: bool = True
    bin_hints: bool = True
    prune_tau: float = 0.0         # bin edges with exp(-maxRatio) |phi_b| below this are left out (0: none)


@dataclasses.dataclass
class FilterSpec:
    """Polynomial of the refinement operator: out = sum_b alpha_b T^{k_b} X."""
    ks: tuple = (4,)
    alphas: tuple = (1.0,)
    sigma: float = 0.0             # self-loop weight (Section IV, A_sigma = A + sigma I)
    lambda_mode: str = "gershgorin"  # or "fixed"
    lambda_fixed: float = 2.0


# ---------------------------------------------------------------------------
# Graph construction
# ---------------------------------------------------------------------------

def node_kinds(nl):
    f = nl["node_flags"].astype(np.int64)
    fixed = (f & FLAG_FIXED) != 0
    macro = (f & FLAG_MACRO) != 0
    std_movable = (~fixed) & (~macro)
    return fixed, macro, std_movable


def expand_macro_pins(nl, params: HintParams):
    """Section V, "Macro pin expansion": every pin sitting on a FIXED macro
    becomes its own fixed node (numbered after the instances, in pin order);
    the net is re-pointed to it.  Movable macros are not expanded.

    Returns (pin node after expansion, owner macro of each new node, pin
    index of each new node)."""
    n_inst = nl["n_inst"]
    pin_node = nl["pin_node"].astype(np.int64)
    fixed, macro, _ = node_kinds(nl)
    if not params.expand_macro_pins:
        return pin_node.copy(), np.zeros(0, np.int64), np.zeros(0, np.int64)
    on_fixed_macro = fixed[pin_node] & macro[pin_node]
    which = np.flatnonzero(on_fixed_macro)
    new_node = pin_node.copy()
    new_node[which] = n_inst + np.arange(which.size)
    return new_node, pin_node[which], which


def net_edges(nl, pin_node_x, first_star_id, clique_max):
    """Weighted expansion of every net into pairwise edges (reading R1).

    The paper treats each net as edges of the graph (Section IV) and scores
    the placement by the weighted quadratic sum over pairs (eq. "Wirelength
    objective") without fixing the net model.  Reading: a net with p pins and
    weight w is a clique of weight w/(p-1) per pin pair if p <= clique_max,
    else a star through a new (movable) node with weight w p/(p-1) per spoke;
    the star's Schur complement is exactly that clique.  Weights are integers
    q = round_half_even(2^32 * weight), evaluated in float64 as
    (2^32 w)/(p-1) for cliques and ((2^32 w) p)/(p-1) for spokes.

    Returns directed COO entries (row, col, q) with duplicates, and the net id
    of each star node."""
    net_ptr = nl["net_ptr"].astype(np.int64)
    deg = np.diff(net_ptr)
    net_w = nl.get("net_w")
    w = np.ones(deg.size) if net_w is None else net_w.astype(np.float32).astype(np.float64)
    rows, cols, qs = [], [], []
    # cliques, grouped by degree
    for p in range(2, clique_max + 1):
        nets = np.flatnonzero(deg == p)
        if nets.size == 0:
            continue
        pins = pin_node_x[net_ptr[nets][:, None] + np.arange(p)[None, :]]      # [n, p]
        q = np.rint((w[nets] * Q_SCALE) / (p - 1)).astype(np.int64)
        for a in range(p):
            for b in range(p):
                if a == b:
                    continue
                r, c = pins[:, a], pins[:, b]
                keep = r != c          # a pair of pins on one node is no edge
                rows.append(r[keep])
                cols.append(c[keep])
                qs.append(q[keep])
    # stars
    star_nets = np.flatnonzero(deg > clique_max)
    star_id = first_star_id + np.arange(star_nets.size)
    if star_nets.size:
        p = deg[star_nets]
        q = np.rint(((w[star_nets] * Q_SCALE) * p) / (p - 1)).astype(np.int64)
        pin_net = np.repeat(np.arange(star_nets.size), p)
        pin_idx = np.concatenate([np.arange(net_ptr[e], net_ptr[e + 1]) for e in star_nets])
        a = pin_node_x[pin_idx]
        z = star_id[pin_net]
        qq = q[pin_net]
        rows += [a, z]
        cols += [z, a]
        qs += [qq, qq]
    if rows:
        return (np.concatenate(rows), np.concatenate(cols), np.concatenate(qs), star_nets)
    e = np.zeros(0, np.int64)
    return e, e, e, star_nets


def canonical_csr_int(rows, cols, q, n):
    """Merge duplicate (row, col) entries by exact int64 sums (reading R2) and
    lay them out row by row with columns ascending (the canonical CSR)."""
    key = rows * np.int64(n) + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    qq = q[order]
    if key.size:
        first = np.concatenate([[True], key[1:] != key[:-1]])
        starts = np.flatnonzero(first)
        qsum = np.add.reduceat(qq, starts)
        ukey = key[starts]
    else:
        qsum = np.zeros(0, np.int64)
        ukey = np.zeros(0, np.int64)
    r = ukey // n
    c = ukey % n
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=row_ptr[1:])
    return row_ptr, c.astype(np.int64), qsum.astype(np.int64)


def base_weight(row_ptr, q):
    """Section V: baseWeight_i is the mean weight of the netlist edges incident
    to i (reading R9: counted after merging parallel edges)."""
    n = row_ptr.size - 1
    nnz = np.diff(row_ptr)
    qdeg = np.zeros(n, np.int64)
    rows = np.flatnonzero(nnz > 0)
    if rows.size:
        qdeg[rows] = np.add.reduceat(q, row_ptr[rows])     # exact int64 row sums
    bw = np.zeros(n)
    nz = nnz > 0
    bw[nz] = (qdeg[nz].astype(np.float64) / Q_SCALE) / nnz[nz]
    return qdeg, nnz, bw


@dataclasses.dataclass
class BinGrid:
    nbx: int
    nby: int
    xl: float
    yl: float
    bw: float      # float64 bin width
    bh: float
    bw32: np.float32
    bh32: np.float32
    xl32: np.float32
    yl32: np.float32


def bin_grid(die, nbx, nby):
    """Section V, "Bin virtual node": numBin_x x numBin_y bins tile the die."""
    d32 = np.asarray(die, np.float32)
    d = d32.astype(np.float64)
    bw32 = np.float32((d32[2] - d32[0]) / np.float32(nbx))
    bh32 = np.float32((d32[3] - d32[1]) / np.float32(nby))
    return BinGrid(nbx, nby, d[0], d[1], (d[2] - d[0]) / nbx, (d[3] - d[1]) / nby,
                   bw32, bh32, d32[0], d32[1])


def cell_bin(grid: BinGrid, x32, y32):
    """Bin of a point, decided in float32: clamp(floor((x - xl) / bw))."""
    fx = np.floor((x32.astype(np.float32) - grid.xl32) / grid.bw32)
    fy = np.floor((y32.astype(np.float32) - grid.yl32) / grid.bh32)
    bx = np.clip(fx, 0, grid.nbx - 1).astype(np.int64)
    by = np.clip(fy, 0, grid.nby - 1).astype(np.int64)
    return bx, by


def bin_density(nl, grid: BinGrid, pos32, macro_ids):
    """Section V: D_b, the current density of bin b (reading R7): the area of
    the movable standard cells whose centre lies in b plus the exact area of
    every macro footprint inside b, over the bin area."""
    _, _, std = node_kinds(nl)
    size = nl["node_size"].astype(np.float64)
    area = np.zeros(grid.nbx * grid.nby)
    cells = np.flatnonzero(std)
    bx, by = cell_bin(grid, pos32[cells, 0], pos32[cells, 1])
    np.add.at(area, by * grid.nbx + bx, size[cells, 0] * size[cells, 1])
    xs = grid.xl + np.arange(grid.nbx + 1) * grid.bw
    ys = grid.yl + np.arange(grid.nby + 1) * grid.bh
    for m in macro_ids:
        cx, cy = float(pos32[m, 0]), float(pos32[m, 1])
        w, h = size[m]
        ox = np.clip(np.minimum(cx + w / 2, xs[1:]) - np.maximum(cx - w / 2, xs[:-1]), 0, None)
        oy = np.clip(np.minimum(cy + h / 2, ys[1:]) - np.maximum(cy - h / 2, ys[:-1]), 0, None)
        area += np.outer(oy, ox).ravel()
    return area / (grid.bw * grid.bh)


def phi(D, C, mu):
    """Section V: phi_b = 2 sigmoid(mu (D_b - C)) - 1."""
    return 2.0 / (1.0 + np.exp(-mu * (D - C))) - 1.0


def window_half(ratio, nb):
    """Section V: n = max(1, floor(0.1 numBin)); reading R8: the window spans
    +-floor(n/2) bins around the centre bin (n odd: exactly n bins)."""
    n = max(1, int(np.floor(np.float32(ratio) * np.float32(nb))))
    return n // 2


def bin_hint_edges(nl, grid: BinGrid, pos32, hint_cells, bw_cell, phis, ratio, first_bin_id, prune_tau=0.0):
    """Section V, "Bin virtual node with density-aware signed edges": every
    hint cell i and every bin b whose window holds i's bin get the edge
    w = -exp(-maxRatio_{i,b}) phi_b baseWeight_i, maxRatio measured from the
    bin centre in units of the half bin size (reading R5: hint cells are the
    movable standard cells with a netlist edge).

    Section IX, "Further speedups", proposes sparsifying the signed
    Laplacian down to its most salient edges.  Reading: an edge's salience is
    its weight relative to the cell's baseWeight, exp(-maxRatio) |phi_b|, and
    with prune_tau > 0 the bin edges of salience below prune_tau are left out
    (macro edges, of salience at least e^-1, always stay)."""
    hx = window_half(ratio, grid.nbx)
    hy = window_half(ratio, grid.nby)
    bx, by = cell_bin(grid, pos32[hint_cells, 0], pos32[hint_cells, 1])
    x = pos32[hint_cells, 0].astype(np.float64)
    y = pos32[hint_cells, 1].astype(np.float64)
    rows, cols, vals = [], [], []
    for dy in range(-hy, hy + 1):
        for dx in range(-hx, hx + 1):
            tx, ty = bx + dx, by + dy
            ok = (tx >= 0) & (tx < grid.nbx) & (ty >= 0) & (ty < grid.nby)
            i = hint_cells[ok]
            b = ty[ok] * grid.nbx + tx[ok]
            xb = grid.xl + (tx[ok] + 0.5) * grid.bw
            yb = grid.yl + (ty[ok] + 0.5) * grid.bh
            ratio_ib = np.maximum(np.abs(x[ok] - xb) / (grid.bw / 2), np.abs(y[ok] - yb) / (grid.bh / 2))
            e = np.exp(-ratio_ib)
            if prune_tau > 0:
                keep = e * np.abs(phis[b]) >= prune_tau
                i, b, e = i[keep], b[keep], e[keep]
            w = -e * phis[b] * bw_cell[i]
            rows.append(i)
            cols.append(first_bin_id + b)
            vals.append(w)
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)


def macro_hint_edges(nl, pos32, hint_cells, bw_cell, macro_ids, first_macro_id):
    """Section V, "Macro virtual node with repulsive (negative) edges": each
    movable hint cell whose centre lies in macro m's closed footprint (reading
    R6; tested in float32) gets w = -exp(-maxRatio_{i,m}) baseWeight_i.

    Candidates are the cells whose x lies within the footprint's x-span plus a
    margin (found on the cells sorted by x); the float32 test then decides."""
    size = nl["node_size"]
    x32 = pos32[hint_cells, 0].astype(np.float32)
    y32 = pos32[hint_cells, 1].astype(np.float32)
    order = np.argsort(x32, kind="stable")
    xs = x32[order].astype(np.float64)
    rows, cols, vals = [], [], []
    for k, m in enumerate(macro_ids):
        mx, my = np.float32(pos32[m, 0]), np.float32(pos32[m, 1])
        hw, hh = np.float32(size[m, 0]) * np.float32(0.5), np.float32(size[m, 1]) * np.float32(0.5)
        margin = 1e-3 * (1.0 + abs(float(mx)) + float(hw))
        lo = np.searchsorted(xs, float(mx) - float(hw) - margin, side="left")
        hi = np.searchsorted(xs, float(mx) + float(hw) + margin, side="right")
        cand = order[lo:hi]
        inside = (np.abs(x32[cand] - mx) <= hw) & (np.abs(y32[cand] - my) <= hh)
        i = np.sort(hint_cells[cand[inside]])
        if i.size == 0:
            continue
        dx = np.abs(pos32[i, 0].astype(np.float64) - float(mx))
        dy = np.abs(pos32[i, 1].astype(np.float64) - float(my))
        ratio_im = np.maximum(dx / (float(size[m, 0]) / 2), dy / (float(size[m, 1]) / 2))
        rows.append(i)
        cols.append(np.full(i.size, first_macro_id + k, np.int64))
        vals.append(-np.exp(-ratio_im) * bw_cell[i])
    if not rows:
        e = np.zeros(0, np.int64)
        return e, e, np.zeros(0)
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)


@dataclasses.dataclass
class Graph:
    """The augmented signed graph of one placement."""
    n_inst: int
    n_tot: int
    first_mpin: int
    first_star: int
    first_mvirt: int
    first_bvirt: int
    mpin_owner: np.ndarray     # macro instance of each macro pin node
    mpin_pin: np.ndarray       # pin index of each macro pin node
    star_net: np.ndarray       # net of each star node
    macro_ids: np.ndarray      # instance id of each macro virtual node
    grid: BinGrid | None
    net_row_ptr: np.ndarray    # canonical netlist CSR (int64 weights q)
    net_col: np.ndarray
    net_q: np.ndarray
    qdeg: np.ndarray
    base_weight: np.ndarray
    hint_row_ptr: np.ndarray   # canonical hint CSR (float64 weights)
    hint_col: np.ndarray
    hint_val: np.ndarray
    phi: np.ndarray | None
    density: np.ndarray | None
    pinned: np.ndarray         # rows overwritten by their input after filtering

    def adjacency(self) -> sp.csr_matrix:
        """Signed weighted adjacency A (float64, symmetric)."""
        n = self.n_tot
        an = sp.csr_matrix((self.net_q.astype(np.float64) / Q_SCALE, self.net_col, self.net_row_ptr), shape=(n, n))
        ah = sp.csr_matrix((self.hint_val, self.hint_col, self.hint_row_ptr), shape=(n, n))
        return (an + ah).tocsr()


def build_netlist_part(nl, params: HintParams):
    """Section V, macro pin expansion + net expansion (reading R1)."""
    n_inst = nl["n_inst"]
    pin_x, mp_owner, mp_pin = expand_macro_pins(nl, params)
    first_star = n_inst + mp_owner.size
    rows, cols, q, star_net = net_edges(nl, pin_x, first_star, params.clique_max)
    return pin_x, mp_owner, mp_pin, first_star, star_net, rows, cols, q


def build_graph(nl, params: HintParams, pos32):
    """BuildLap of Algorithm 1 (Section V): the netlist graph with its area
    hints for the placement ``pos32`` (float32, [n_inst, 2])."""
    n_inst = nl["n_inst"]
    fixed, macro, std = node_kinds(nl)
    pin_x, mp_owner, mp_pin, first_star, star_net, rows, cols, q = build_netlist_part(nl, params)
    first_mvirt = first_star + star_net.size
    macro_ids = np.flatnonzero(macro) if params.macro_hints else np.zeros(0, np.int64)
    first_bvirt = first_mvirt + macro_ids.size
    nbins = params.nbx * params.nby if params.bin_hints else 0
    n_tot = first_bvirt + nbins

    row_ptr, col, qv = canonical_csr_int(rows, cols, q, n_tot)
    qdeg, nnz, bw_cell = base_weight(row_ptr, qv)

    pos32 = np.asarray(pos32, np.float32)
    hint_cells = np.flatnonzero(std & (qdeg[:n_inst] > 0))
    hr, hc, hv = [], [], []
    grid = None
    ph = dens = None
    if params.macro_hints and macro_ids.size:
        r, c, v = macro_hint_edges(nl, pos32, hint_cells, bw_cell, macro_ids, first_mvirt)
        hr += [r, c]; hc += [c, r]; hv += [v, v]
    if params.bin_hints:
        grid = bin_grid(nl["die"], params.nbx, params.nby)
        all_macros = np.flatnonzero(macro)
        dens = bin_density(nl, grid, pos32, all_macros)
        ph = phi(dens, params.bin_capacity, params.mu)
        r, c, v = bin_hint_edges(nl, grid, pos32, hint_cells, bw_cell, ph,
                                 params.detection_ratio, first_bvirt, params.prune_tau)
        hr += [r, c]; hc += [c, r]; hv += [v, v]
    if hr:
        hr, hc, hv = np.concatenate(hr), np.concatenate(hc), np.concatenate(hv)
        order = np.lexsort((hc, hr))
        hr, hc, hv = hr[order], hc[order], hv[order]
    else:
        hr = hc = np.zeros(0, np.int64)
        hv = np.zeros(0)
    hint_row_ptr = np.zeros(n_tot + 1, np.int64)
    np.cumsum(np.bincount(hr, minlength=n_tot), out=hint_row_ptr[1:])

    pinned = np.zeros(n_tot, bool)
    pinned[:n_inst] = fixed
    pinned[n_inst:first_star] = True      # macro pin nodes
    pinned[first_mvirt:] = True           # virtual nodes
    return Graph(n_inst, n_tot, n_inst, first_star, first_mvirt, first_bvirt,
                 mp_owner, mp_pin, star_net, macro_ids, grid,
                 row_ptr, col, qv, qdeg, bw_cell, hint_row_ptr, hc, hv, ph, dens, pinned)


# ---------------------------------------------------------------------------
# Operator and filter
# ---------------------------------------------------------------------------

def operator(g: Graph, sigma=0.0, lambda_mode="gershgorin", lambda_fixed=2.0):
    """Signed normalised Laplacian and the refinement operator.

    Section II-A: L~ = D^{-1/2} (D - A) D^{-1/2}; Section IV: A_sigma = A + sigma I.
    Reading R3: on a signed graph the degree is the absolute one,
    d_i = sum_j |A_ij|, so that D - A stays positive semi-definite.
    Reading R12: a row with d_i + sigma = 0 is left alone (L_ii = 0).
    Section V: lambda_up is the Gershgorin bound max_i (L_ii + sum_j |L_ij|),
    and T = (lambda_up I - L)/lambda_up = I - L/lambda_up.

    Returns (L, T, d, s, lambda_up) with L, T scipy CSR (float64)."""
    A = g.adjacency()
    n = g.n_tot
    d = np.asarray(abs(A).sum(axis=1)).ravel() + sigma
    s = np.zeros(n)
    nz = d > 0
    s[nz] = 1.0 / np.sqrt(d[nz])
    S = sp.diags(s)
    L = (sp.diags(nz.astype(np.float64)) - S @ (A + sigma * sp.identity(n)) @ S).tocsr()
    if lambda_mode == "gershgorin":
        absL = abs(L)
        diag = L.diagonal()
        lam = float(np.max(np.abs(diag) + (np.asarray(absL.sum(axis=1)).ravel() - np.abs(diag)))) if n else 0.0
    else:
        lam = float(lambda_fixed)
    if lam == 0.0:
        T = sp.identity(n, format="csr")
    else:
        T = (sp.identity(n) - L / lam).tocsr()
    return L, T, d, s, lam


def expand_signal(nl, g: Graph, G):
    """Values of the nodes added by the construction (reading R10): a macro pin
    node sits at its macro's centre plus the pin offset, a star node at the
    mean of its pins' node values, a macro virtual node at the macro centre, a
    bin virtual node at the bin centre.  Even columns are x, odd columns y."""
    G = np.asarray(G, np.float64)
    C = G.shape[1]
    X = np.zeros((g.n_tot, C))
    X[:g.n_inst] = G
    off = nl["pin_off"].astype(np.float64)
    xy = np.arange(C) % 2
    if g.mpin_owner.size:
        X[g.first_mpin:g.first_star] = G[g.mpin_owner] + off[g.mpin_pin][:, xy]
    if g.star_net.size:
        net_ptr = nl["net_ptr"].astype(np.int64)
        node_x = _expanded_pin_nodes(nl, g)
        for k, e in enumerate(g.star_net):
            X[g.first_star + k] = X[node_x[net_ptr[e]:net_ptr[e + 1]]].mean(axis=0)
    if g.macro_ids.size:
        X[g.first_mvirt:g.first_bvirt] = G[g.macro_ids]
    if g.grid is not None:
        gr = g.grid
        b = np.arange(gr.nbx * gr.nby)
        cx = gr.xl + (b % gr.nbx + 0.5) * gr.bw
        cy = gr.yl + (b // gr.nbx + 0.5) * gr.bh
        X[g.first_bvirt:, 0::2] = cx[:, None]
        X[g.first_bvirt:, 1::2] = cy[:, None]
    return X


def _expanded_pin_nodes(nl, g: Graph):
    node = nl["pin_node"].astype(np.int64).copy()
    if g.mpin_pin.size:
        node[g.mpin_pin] = g.first_mpin + np.arange(g.mpin_pin.size)
    return node


def apply_filter(nl, g: Graph, spec: FilterSpec, G, return_full=False, pin=True):
    """Apply the polynomial filter.

    H = sum_b alpha_b T^{k_b} applied to the expanded signal (Section V eq.
    "refine-filter"; the three-band bank of Section IV eq. "GiFt filter" on the
    signed operator, reading R13), then every fixed or virtual row is reset to
    its input (Section IV: re-pin fixed objects after filtering; reading R11:
    once, after the whole polynomial).  Returns the instance rows."""
    _, T, _, _, lam = operator(g, spec.sigma, spec.lambda_mode, spec.lambda_fixed)
    X = expand_signal(nl, g, G)
    kmax = max(spec.ks) if spec.ks else 0
    out = np.zeros_like(X)
    Y = X.copy()
    for j in range(0, kmax + 1):
        if j > 0:
            Y = T @ Y
        for k, a in zip(spec.ks, spec.alphas):
            if k == j:
                out += a * Y
    if pin:
        out[g.pinned] = X[g.pinned]
    if return_full:
        return out, lam
    return out[:g.n_inst]


def refine(nl, params: HintParams, spec: FilterSpec, G0, T_hint, gamma):
    """Algorithm 1 (Section V): for each round, build L_hint from the current
    placement (column pair 0), filter every column with H_r, and relax
    g <- (1 - gamma) g + gamma g~ on movable rows; fixed rows stay as given."""
    fixed, _, _ = node_kinds(nl)
    G = np.asarray(G0, np.float64).copy()
    G32 = np.asarray(G0, np.float32)
    for _ in range(T_hint):
        g = build_graph(nl, params, G32[:, :2])
        Gt = apply_filter(nl, g, spec, G)
        Gn = (1.0 - gamma) * G + gamma * Gt
        Gn[fixed] = G[fixed]
        G = Gn
        G32 = G.astype(np.float32)
    return G


def hpwl(nl, G):
    """Half-perimeter wirelength of every net and its total, per (x, y) column
    pair: sum over nets of (max - min) of the pin x plus that of the pin y,
    pin position = node position + pin offset (original, unexpanded pins)."""
    G = np.asarray(G, np.float64)
    net_ptr = nl["net_ptr"].astype(np.int64)
    pin_node = nl["pin_node"].astype(np.int64)
    off = nl["pin_off"].astype(np.float64)
    deg = np.diff(net_ptr)
    nonempty = deg > 0
    starts = net_ptr[:-1][nonempty]
    per_net = np.zeros((deg.size, G.shape[1] // 2))
    for c in range(G.shape[1] // 2):
        px = G[pin_node, 2 * c] + off[:, 0]
        py = G[pin_node, 2 * c + 1] + off[:, 1]
        hx = np.maximum.reduceat(px, starts) - np.minimum.reduceat(px, starts)
        hy = np.maximum.reduceat(py, starts) - np.minimum.reduceat(py, starts)
        per_net[nonempty, c] = hx + hy
    return per_net.sum(axis=0), per_net


# ---------------------------------------------------------------------------
# GiFt: the unsigned multi-band initializer that produces Algorithm 1's input
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class GiftBank:
    """Section IV eq. "GiFt filter": H = sum_b alpha_b Atilde_{sigma_b}^{k_b}.
    The paper's bands are Atilde_2^2 (high), Atilde_4^2 (mid) and Atilde_4^4
    (low), i.e. (k, sigma) = (2, 2), (2, 4), (4, 4); the weights are tuning
    parameters that sum to 1 (Table "Parameter space": the high-band weight is
    1 - low - mid).  The default weights are a reading (none is printed)."""
    ks: tuple = (2, 2, 4)
    sigmas: tuple = (2.0, 4.0, 4.0)
    alphas: tuple = (0.2, 0.3, 0.5)


def gift_operator(g: Graph, sigma):
    """Section IV: A_sigma = A + sigma I, D_sigma = D + sigma I and the
    augmented normalised adjacency Atilde_sigma = D_sigma^-1/2 A_sigma
    D_sigma^-1/2 (eq. "GiFt" for sigma = 0).  Reading R12: a row with
    d_i + sigma = 0 (an isolated node without self-loop) is left unchanged,
    which is also what Atilde_sigma does to an isolated node for sigma > 0."""
    A = g.adjacency()
    n = g.n_tot
    d = np.asarray(A.sum(axis=1)).ravel() + sigma
    s = np.zeros(n)
    nz = d > 0
    s[nz] = 1.0 / np.sqrt(d[nz])
    At = sp.diags(s) @ (A + sigma * sp.identity(n)) @ sp.diags(s)
    return (At + sp.diags((~nz).astype(np.float64))).tocsr()


def gift(nl, g: Graph, bank: GiftBank, G, pin=True, return_full=False):
    """GSP-based initialization (Section IV, steps 2-3): the bank applied to
    the expanded signal (the instance graph's added star nodes carry the mean
    of their pins, reading R10), then every fixed row reset to its input.
    The graph must carry no area hints (GiFt runs before them)."""
    assert g.hint_val.size == 0, "GiFt filters the netlist graph (no area hints)"
    X = expand_signal(nl, g, G)
    out = np.zeros_like(X)
    for k, sigma, a in zip(bank.ks, bank.sigmas, bank.alphas):
        At = gift_operator(g, sigma)
        Y = X.copy()
        for _ in range(k):
            Y = At @ Y
        out += a * Y
    if pin:
        out[g.pinned] = X[g.pinned]
    return out if return_full else out[:g.n_inst]
