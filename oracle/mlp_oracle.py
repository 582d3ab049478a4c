"""FP64 oracle of the learned surrogate of the refinement filter.

TEST INFRASTRUCTURE ONLY (see ahr_oracle.py): nothing in the product path
imports it.

The surrogate is a project addition, not part of the paper: it approximates
the order-K signed filter of Section V (eq. "refine-filter", banked as in
Section IV eq. "GiFt filter") from the input and three low-order powers of
the same operator T.  For every movable instance row i and column c:

    h_j   = (T^j X)[i, c],  j = 0, 1, 2, 3       (the unpinned chain; h_0 = X)
    m_c, s_c = mean and standard deviation of h_3[:, c] over movable rows
    r_c   = root mean square of (h_0 - h_3)[:, c] over movable rows
    f     = [(h_0 - h_3)/r_c, (h_1 - h_3)/r_c, (h_2 - h_3)/r_c, (h_3 - m_c)/s_c,
             log1p(d_i), hsum_i / d_i, log(s_c / r_c)]
                                                 (hsum_i = sum of row i's hint weights)
    o     = w3 . relu(W2 relu(W1 f + b1) + b2) + b3
    y_hat = beta_0 h_0 + beta_1 h_1 + beta_2 h_2 + beta_3 h_3 + r_c o

r_c is the displacement of three hops, a length set by the graph's local
neighbourhoods; s_c grows with the die.  Scaling the differences of hops and
the network's output by r_c keeps them the same size on netlists of any
size, and log(s_c / r_c), one value per column, tells the network how the
two lengths compare.  A column with s_c = 0 or r_c = 0 takes 1 in its place.

The GPU evaluates the network with bfloat16 operands (features, weights and
hidden activations rounded to nearest-even bfloat16) and float32
accumulation; this oracle rounds at the same points and accumulates in
float64.  Training minimises the mean of (o - r)^2 with
r = (y_ref - sum_j beta_j h_j) / r_c; gradients pass straight through the
rounding.
"""
from __future__ import annotations

import numpy as np

from . import ahr_oracle as O

HIDDEN = 64
NFEAT = 7
NHOPS = 4        # h_0 .. h_3
FEAT_PAD = 8


# flat float32 parameter vector: W1[64][8], b1[64], W2[64][64], b2[64], w3[64], b3
def layout():
    off = {}
    k = 0
    for name, size in (("W1", HIDDEN * FEAT_PAD), ("b1", HIDDEN), ("W2", HIDDEN * HIDDEN), ("b2", HIDDEN),
                       ("w3", HIDDEN), ("b3", 1)):
        off[name] = (k, size)
        k += size
    return off, k


OFFSETS, NPARAM = layout()


def unpack(p):
    p = np.asarray(p, np.float64)
    g = lambda n: p[OFFSETS[n][0]:OFFSETS[n][0] + OFFSETS[n][1]]
    return (g("W1").reshape(HIDDEN, FEAT_PAD), g("b1"), g("W2").reshape(HIDDEN, HIDDEN), g("b2"), g("w3"),
            g("b3")[0])


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.asarray(W1).ravel(), b1, np.asarray(W2).ravel(), b2, w3, [b3]]).astype(np.float64)


def init_params(seed=0):
    """He-style initial weights (the trainer's starting point; W1 columns for
    the padding features are zero)."""
    rng = np.random.default_rng(seed)
    W1 = np.zeros((HIDDEN, FEAT_PAD))
    W1[:, :NFEAT] = rng.normal(0, np.sqrt(2.0 / NFEAT), (HIDDEN, NFEAT))
    W2 = rng.normal(0, np.sqrt(2.0 / HIDDEN), (HIDDEN, HIDDEN))
    w3 = rng.normal(0, np.sqrt(1.0 / HIDDEN), HIDDEN)
    return pack(W1, np.zeros(HIDDEN), W2, np.zeros(HIDDEN), w3, 0.0).astype(np.float32)


def bf16(x):
    """Round float32 values to the nearest bfloat16 (ties to even); returned
    as float64 holding the exact bfloat16 value."""
    a = np.ascontiguousarray(np.asarray(x, np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def hops(nl, g: O.Graph, G, sigma=0.0, lambda_mode="gershgorin", lambda_fixed=2.0, k=3):
    """h_j = T^j X for j = 0..k on the extended signal (no pinning; h_0 = X)."""
    _, T, d, _, _ = O.operator(g, sigma, lambda_mode, lambda_fixed)
    Y = O.expand_signal(nl, g, G)
    out = [Y]
    for _ in range(k):
        Y = T @ Y
        out.append(Y)
    return out, d


def hint_sum(g: O.Graph):
    """Signed sum of each row's hint weights."""
    n = g.n_tot
    rows = np.repeat(np.arange(n), np.diff(g.hint_row_ptr))
    return np.bincount(rows, weights=g.hint_val, minlength=n)


def column_stats(h0, h3, mov):
    """m_c and s_c (mean and standard deviation of h_3) and r_c (root mean
    square of h_0 - h_3), over the movable rows; a zero s_c or r_c becomes 1."""
    m = h3[mov].mean(axis=0)
    s = h3[mov].std(axis=0)
    r = np.sqrt(np.mean((h0[mov] - h3[mov]) ** 2, axis=0))
    return m, np.where(s > 0, s, 1.0), np.where(r > 0, r, 1.0)


def features(nl, g: O.Graph, G, sigma=0.0, lambda_mode="gershgorin", lambda_fixed=2.0):
    """Features of every (instance row, column) and the column statistics.

    Returns (F [n_inst, C, 7], (h0, h1, h2, h3) [n_inst, C], (m, s, r) [C])."""
    hs, d = hops(nl, g, G, sigma, lambda_mode, lambda_fixed)
    n = g.n_inst
    h0, h1, h2, h3 = (h[:n] for h in hs)
    mov = (nl["node_flags"] & O.FLAG_FIXED) == 0
    m, s, r = column_stats(h0, h3, mov)
    dd = d[:n]
    hs_ = hint_sum(g)[:n]
    C = h1.shape[1]
    F = np.zeros((n, C, NFEAT))
    F[:, :, 0] = (h0 - h3) / r
    F[:, :, 1] = (h1 - h3) / r
    F[:, :, 2] = (h2 - h3) / r
    F[:, :, 3] = (h3 - m) / s
    F[:, :, 4] = np.log1p(dd)[:, None]
    F[:, :, 5] = np.where(dd > 0, hs_ / np.where(dd > 0, dd, 1.0), 0.0)[:, None]
    F[:, :, 6] = np.log(s / r)[None, :]
    return F, (h0, h1, h2, h3), (m, s, r)


def forward(params, F, rounding=True):
    """o for each feature row F [N, 5]; returns (o, cache).  rounding=False
    keeps every operand exact (used to pin the gradient by finite
    differences)."""
    q = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    W1, b1, W2, b2, w3, b3 = unpack(params)
    x = np.zeros((F.shape[0], FEAT_PAD))
    x[:, :NFEAT] = F
    xq = q(x)
    W1q, W2q, w3q = q(W1), q(W2), q(w3)
    b1f, b2f = (np.float32(b1).astype(np.float64), np.float32(b2).astype(np.float64)) if rounding else (b1, b2)
    z1 = xq @ W1q.T + b1f
    a1 = np.maximum(z1, 0)
    a1q = q(a1)
    z2 = a1q @ W2q.T + b2f
    a2 = np.maximum(z2, 0)
    a2q = q(a2)
    o = a2q @ w3q + (float(np.float32(b3)) if rounding else b3)
    return o, (xq, z1, a1q, z2, a2q, W2q, w3q)


def loss_grad(params, F, r, rounding=True):
    """Mean squared error of o against r, and its gradient with respect to
    the float32 parameters (straight through the bfloat16 rounding)."""
    o, (xq, z1, a1q, z2, a2q, W2q, w3q) = forward(params, F, rounding)
    N = F.shape[0]
    e = o - r
    loss = float(np.mean(e * e))
    do = 2.0 * e / N
    gw3 = a2q.T @ do
    gb3 = do.sum()
    dz2 = np.outer(do, w3q) * (z2 > 0)
    gW2 = dz2.T @ a1q
    gb2 = dz2.sum(axis=0)
    da1 = dz2 @ W2q
    dz1 = da1 * (z1 > 0)
    gW1 = dz1.T @ xq
    gb1 = dz1.sum(axis=0)
    return loss, pack(gW1, gb1, gW2, gb2, gw3, gb3)


def predict(params, beta, F, h, r):
    """y_hat [n_inst, C] from features F [n_inst, C, 7], hops h = (h0..h3)
    and the local scale r [C]."""
    n, C, _ = F.shape
    o, _ = forward(params, F.reshape(n * C, NFEAT))
    o = o.reshape(n, C)
    return sum(beta[j] * h[j] for j in range(NHOPS)) + r[None, :] * o


def learned_filter(nl, g, params, beta, G, sigma=0.0, lambda_mode="gershgorin", lambda_fixed=2.0):
    """The surrogate's output on the instance rows (fixed rows keep their input)."""
    F, h, (m, s, r) = features(nl, g, G, sigma, lambda_mode, lambda_fixed)
    y = predict(params, beta, F, h, r)
    fixed = (nl["node_flags"] & O.FLAG_FIXED) != 0
    y[fixed] = np.asarray(G, np.float64)[fixed]
    return y
