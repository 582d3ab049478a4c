"""Seeded synthetic mixed-size netlists and initial placement signals.

This module only draws inputs.  It holds none of the method's arithmetic:
no net expansion, no hint edges, no filtering.  Both the CPU oracle and the
HIP library consume exactly the arrays it returns.

Shapes follow the paper's benchmark table (Section VI, Table "benchmark
characteristics"): cells ~ nets, fixed objects 0.1-4 % of instances.  The
recipe (units, die, macros, degree mix, pin locality, initial signal) is
stated in ``generate``'s docstring.

Arrays (all numpy, little-endian):
  node_flags  uint8[N]     bit0 FIXED, bit1 MACRO
  node_size   float32[N,2] (w, h)
  net_ptr     int32[E+1]
  pin_node    int32[P]     instance id of each pin
  pin_off     float32[P,2] pin offset from the instance centre
  die         float32[4]   (xl, yl, xh, yh)
  g0          float32[N,C] initial signal; fixed rows hold the fixed position
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

FIXED = 1
MACRO = 2


@dataclasses.dataclass(frozen=True)
class NetlistConfig:
    name: str
    n_std: int
    n_macro: int
    n_io: int
    n_nets: int
    movable_macros: bool
    macro_side_min: float      # rows
    macro_side_max: float      # rows
    macro_area_frac: float     # target macro share of total area (<=0: unscaled sides)
    big_frac: float            # share of nets drawn log-uniform in [big_min, big_max]
    big_min: int
    big_max: int
    ncols: int                 # signal columns (pairs of x, y)
    seed: int


# Configurations named by workload and size.
TINY = NetlistConfig("tiny-2k", 2000, 8, 32, 2200, True, 20, 60, -1.0,
                     0.0, 51, 51, 2, 101)
MID = NetlistConfig("mid-210k", 210_000, 500, 1200, 220_000, False, 10, 200, 0.40,
                    0.005, 51, 2000, 4, 202)
LARGE = NetlistConfig("large-2.2M", 2_200_000, 8000, 8000, 2_250_000, False, 10, 200,
                      0.40, 0.0001, 51, 10_000, 4, 505)


def small(n_std: int, seed: int, ncols: int = 2, n_macro: int | None = None,
          n_io: int | None = None, movable_macros: bool = False,
          big_frac: float = 0.0) -> NetlistConfig:
    """A scaled-down configuration for parity tests (several tiles, ragged)."""
    if n_macro is None:
        n_macro = max(2, n_std // 100)
    if n_io is None:
        n_io = max(4, n_std // 150)
    return NetlistConfig(f"small-{n_std}-{seed}", n_std, n_macro, n_io,
                         int(n_std * 1.05), movable_macros, 6, 40, 0.30,
                         big_frac, 51, max(52, n_std // 20), ncols, seed)


def batch_member(n_std: int, seed: int, macro_pct: float) -> NetlistConfig:
    """One netlist of the uneven batched workload (5k-200k cells, 2-5 % macros)."""
    n_macro = max(2, int(round(n_std * macro_pct)))
    n_io = max(8, n_std // 200)
    return NetlistConfig(f"batch-{n_std}-{seed}", n_std, n_macro, n_io,
                         int(n_std * 1.05), False, 4, 80, 0.30,
                         0.002, 51, max(52, min(2000, n_std // 50)), 4, seed)


def sized(n_std: int, seed: int) -> NetlistConfig:
    """A netlist of any size between the mid-210k and large-2.2M shapes: the
    per-cell rates of macros, I/O pins and nets and the big-net mix are
    interpolated in log(size) between the two (clamped outside them)."""
    t = (math.log(n_std) - math.log(MID.n_std)) / (math.log(LARGE.n_std) - math.log(MID.n_std))
    t = min(1.0, max(0.0, t))
    lerp = lambda a, b: (1.0 - t) * a + t * b
    n_macro = int(round(n_std * lerp(MID.n_macro / MID.n_std, LARGE.n_macro / LARGE.n_std)))
    n_io = int(round(n_std * lerp(MID.n_io / MID.n_std, LARGE.n_io / LARGE.n_std)))
    n_nets = int(round(n_std * lerp(MID.n_nets / MID.n_std, LARGE.n_nets / LARGE.n_std)))
    return NetlistConfig(f"sized-{n_std}-{seed}", n_std, max(2, n_macro), max(8, n_io), n_nets, False,
                         MID.macro_side_min, MID.macro_side_max, MID.macro_area_frac,
                         lerp(MID.big_frac, LARGE.big_frac), MID.big_min,
                         int(round(lerp(MID.big_max, LARGE.big_max))), 4, seed)


def batch_sizes(n_graphs: int = 64, lo: int = 5000, hi: int = 200_000,
                seed: int = 3000) -> list[tuple[int, int, float]]:
    """(n_std, seed, macro_pct) of each member of the batched workload."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(math.log(lo), math.log(hi), n_graphs))
    pct = rng.uniform(0.02, 0.05, n_graphs)
    return [(int(s), seed + i, float(p)) for i, (s, p) in enumerate(zip(sizes, pct))]


def _degrees(rng, n, big_frac, big_min, big_max):
    """Net degree mix: 60 % 2-pin, 20 % 3-pin, 17 % U{4..10}, rest U{11..50},
    of which ``big_frac`` (absolute share) is log-uniform in [big_min, big_max]."""
    u = rng.random(n)
    deg = np.empty(n, dtype=np.int64)
    deg[u < 0.60] = 2
    m = (u >= 0.60) & (u < 0.80)
    deg[m] = 3
    m = (u >= 0.80) & (u < 0.97)
    deg[m] = rng.integers(4, 11, m.sum())
    m = u >= 0.97
    deg[m] = rng.integers(11, 51, m.sum())
    if big_frac > 0:
        big = u >= 1.0 - big_frac
        nb = int(big.sum())
        deg[big] = np.floor(np.exp(rng.uniform(math.log(big_min),
                                               math.log(big_max + 1), nb))).astype(np.int64)
        deg[big] = np.clip(deg[big], big_min, big_max)
    return deg


def _draw_pins(rng, deg, n_std, lat_w, lat_h):
    """Pins of each net: an anchor cell, then 90 % locality-biased picks within
    a lattice radius ~2*sqrt(p), 10 % uniform picks; no repeated cell in a net.

    Returns a list of (net ids, pins[n, p]) groups and the anchor of every net.
    """
    anchors = rng.integers(0, n_std, deg.size)
    order = np.argsort(deg, kind="stable")
    sdeg = deg[order]
    bounds = np.flatnonzero(np.diff(sdeg)) + 1
    groups = []
    for g in np.split(order, bounds):
        if g.size == 0:
            continue
        p = int(deg[g[0]])
        if p <= 64:
            groups.append((g, _local_pick(rng, anchors[g], p, n_std, lat_w, lat_h)))
        else:
            for net in g:
                groups.append((np.array([net]),
                               _local_pick(rng, anchors[net:net + 1], p, n_std, lat_w, lat_h)))
    return groups, anchors


def _local_pick(rng, anchors, p, n_std, lat_w, lat_h):
    m = anchors.size
    rad = max(1, int(round(2.0 * math.sqrt(p))))
    ax = anchors % lat_w
    ay = anchors // lat_w
    pins = np.empty((m, p), dtype=np.int64)
    pins[:, 0] = anchors

    def fill(rows, cols):
        k = rows.size
        loc = rng.random(k) < 0.9
        dx = rng.integers(-rad, rad + 1, k)
        dy = rng.integers(-rad, rad + 1, k)
        x = np.clip(ax[rows] + dx, 0, lat_w - 1)
        y = np.clip(ay[rows] + dy, 0, lat_h - 1)
        cand = y * lat_w + x
        cand = np.where(cand >= n_std, rng.integers(0, n_std, k), cand)
        uni = rng.integers(0, n_std, k)
        pins[rows, cols] = np.where(loc, cand, uni)

    rr, cc = np.meshgrid(np.arange(m), np.arange(1, p), indexing="ij")
    fill(rr.ravel(), cc.ravel())
    # redraw repeated cells until every net has distinct pins
    for _ in range(200):
        s = np.sort(pins, axis=1)
        dup_rows = np.flatnonzero((s[:, 1:] == s[:, :-1]).any(axis=1))
        if dup_rows.size == 0:
            break
        sub = pins[dup_rows]
        o = np.argsort(sub, axis=1, kind="stable")
        ss = np.take_along_axis(sub, o, axis=1)
        dupmask_sorted = np.zeros_like(ss, dtype=bool)
        dupmask_sorted[:, 1:] = ss[:, 1:] == ss[:, :-1]
        dupmask = np.zeros_like(dupmask_sorted)
        np.put_along_axis(dupmask, o, dupmask_sorted, axis=1)
        dupmask[:, 0] = False
        r, c = np.nonzero(dupmask)
        fill(dup_rows[r], c)
    else:
        raise RuntimeError("could not draw distinct pins")
    return pins


def _place_fixed_macros(rng, sizes, die_side, max_tries=2000):
    """Non-overlapping positions by seeded rejection sampling on a grid index."""
    half = die_side / 2.0
    n = sizes.shape[0]
    pos = np.zeros((n, 2))
    cell = max(float(sizes.max()), die_side / 256.0)
    ng = int(math.ceil(die_side / cell)) + 1
    grid: dict[tuple[int, int], list[int]] = {}
    order = np.argsort(-(sizes[:, 0] * sizes[:, 1]), kind="stable")
    for m in order:
        w, h = sizes[m]
        for _ in range(max_tries):
            x = rng.uniform(-half + w / 2, half - w / 2)
            y = rng.uniform(-half + h / 2, half - h / 2)
            gx = int((x + half) / cell)
            gy = int((y + half) / cell)
            ok = True
            for ix in range(max(0, gx - 1), min(ng, gx + 2)):
                for iy in range(max(0, gy - 1), min(ng, gy + 2)):
                    for o in grid.get((ix, iy), ()):
                        ox, oy = pos[o]
                        ow, oh = sizes[o]
                        if abs(x - ox) < (w + ow) / 2 and abs(y - oy) < (h + oh) / 2:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if ok:
                pos[m] = (x, y)
                grid.setdefault((gx, gy), []).append(int(m))
                break
        else:
            raise RuntimeError("macro placement failed; die too crowded")
    return pos


def generate(cfg: NetlistConfig) -> dict:
    """Draw one netlist and its initial signal.

    Recipe:
      * units: site width = row height = 1; std cells are w in U{1..4} x 1,
        movable, pins at the cell centre; I/O pins are zero-size, fixed, evenly
        spaced on the die boundary with seeded jitter;
      * die: square, centred on the origin, side = sqrt(total area / 0.70);
      * macros: square-ish (aspect U[0.8, 1.25]), side log-uniform in
        [side_min, side_max]; when ``macro_area_frac`` > 0 all sides are scaled
        by one factor so macros hold that share of the total area; fixed
        macros are placed without overlap; about 0.75 pins per unit of
        perimeter (clamped to [8, 512]) sit on each macro's boundary;
      * nets: degree mix of ``_degrees``; pins are locality-biased in a hidden
        lattice that maps std cells onto the die; every std cell lies on at
        least one net; each macro pin and each I/O joins one net anchored near
        it; instance ids are a seeded random permutation;
      * initial signal: ``ncols/2`` (x, y) column pairs; movable cells sit at
        a centre-concentrated warp of the hidden lattice (normal quantiles,
        sd = die side / 6) plus independent noise of one lattice spacing per
        pair, so connected cells are near each other and crowd the centre --
        the shape of a low-pass (GSP) initial placement; macros (movable or
        fixed) and I/O sit at their drawn positions.
    """
    rng = np.random.default_rng(cfg.seed)
    n_std, n_mac, n_io = cfg.n_std, cfg.n_macro, cfg.n_io
    n_inst = n_std + n_mac + n_io

    std_w = rng.integers(1, 5, n_std).astype(np.float64)
    std_area = float(std_w.sum())

    side = np.exp(rng.uniform(math.log(cfg.macro_side_min), math.log(cfg.macro_side_max), n_mac))
    aspect = rng.uniform(0.8, 1.25, n_mac)
    mw = side * np.sqrt(aspect)
    mh = side / np.sqrt(aspect)
    if cfg.macro_area_frac > 0 and n_mac > 0:
        target = cfg.macro_area_frac / (1.0 - cfg.macro_area_frac) * std_area
        scale = math.sqrt(target / float((mw * mh).sum()))
        mw *= scale
        mh *= scale
    mw = np.maximum(np.round(mw), 2.0)
    mh = np.maximum(np.round(mh), 2.0)
    total_area = std_area + float((mw * mh).sum())
    die_side = math.ceil(math.sqrt(total_area / 0.70))
    half = die_side / 2.0
    die = np.array([-half, -half, half, half], dtype=np.float32)

    msz = np.stack([mw, mh], axis=1)
    if cfg.movable_macros:
        mpos = np.stack([rng.uniform(-half + mw / 2, half - mw / 2),
                         rng.uniform(-half + mh / 2, half - mh / 2)], axis=1)
    else:
        mpos = _place_fixed_macros(rng, msz, die_side)

    # I/O on the boundary
    t = (np.arange(n_io) + rng.uniform(0.2, 0.8, n_io)) / max(n_io, 1) * 4.0
    side_id = np.floor(t).astype(np.int64)
    frac = t - side_id
    iox = np.where(side_id == 0, -half + frac * die_side,
          np.where(side_id == 1, half, np.where(side_id == 2, half - frac * die_side, -half)))
    ioy = np.where(side_id == 0, -half,
          np.where(side_id == 1, -half + frac * die_side, np.where(side_id == 2, half, half - frac * die_side)))
    iopos = np.stack([iox, ioy], axis=1)

    # hidden lattice for std cells (maps onto the die)
    lat_w = int(math.ceil(math.sqrt(n_std)))
    lat_h = int(math.ceil(n_std / lat_w))

    # nets: reserve room for coverage nets
    n_main = max(1, int(cfg.n_nets * 0.97))
    deg = _degrees(rng, n_main, cfg.big_frac, cfg.big_min, cfg.big_max)
    groups, anchors = _draw_pins(rng, deg, n_std, lat_w, lat_h)
    covered = np.zeros(n_std, dtype=bool)
    for _, pins in groups:
        covered[pins.ravel()] = True
    unc = np.flatnonzero(~covered)
    nb = np.where(unc + 1 < n_std, unc + 1, unc - 1)
    n_next = n_main
    if unc.size:
        groups.append((np.arange(n_next, n_next + unc.size), np.stack([unc, nb], axis=1)))
        anchors = np.concatenate([anchors, unc])
        n_next += unc.size
    fill = cfg.n_nets - n_next
    if fill > 0:
        a = rng.integers(0, n_std, fill)
        groups.append((np.arange(n_next, n_next + fill), _local_pick(rng, a, 2, n_std, lat_w, lat_h)))
        anchors = np.concatenate([anchors, a])
        n_next += fill
    n_nets = n_next

    # attach macro pins and I/O to nets anchored near them (std-cell-only nets)
    anc_x = (anchors % lat_w + 0.5) / lat_w * die_side - half
    anc_y = (anchors // lat_w + 0.5) / lat_h * die_side - half
    coarse = max(1, int(math.sqrt(n_nets / 8)))
    cb = (np.clip(((anc_y + half) / die_side * coarse).astype(np.int64), 0, coarse - 1) * coarse
          + np.clip(((anc_x + half) / die_side * coarse).astype(np.int64), 0, coarse - 1))
    net_order = np.argsort(cb, kind="stable")
    cb_sorted = cb[net_order]
    starts = np.searchsorted(cb_sorted, np.arange(coarse * coarse), side="left")
    ends = np.searchsorted(cb_sorted, np.arange(coarse * coarse), side="right")

    def nets_near(px, py):
        b = (np.clip(((py + half) / die_side * coarse).astype(np.int64), 0, coarse - 1) * coarse
             + np.clip(((px + half) / die_side * coarse).astype(np.int64), 0, coarse - 1))
        lo, hi = starts[b], ends[b]
        cnt = hi - lo
        r = rng.random(px.size)
        pick = lo + np.floor(r * np.maximum(cnt, 1)).astype(np.int64)
        pick = np.minimum(pick, len(net_order) - 1)
        res = net_order[pick]
        empty = cnt == 0
        res[empty] = rng.integers(0, n_nets, int(empty.sum()))
        return res

    # macro pins on the boundary
    perim = 2.0 * (mw + mh)
    npin_m = np.clip(np.round(0.75 * perim), 8, 512).astype(np.int64)
    mp_macro = np.repeat(np.arange(n_mac), npin_m)
    s = rng.random(mp_macro.size) * perim[mp_macro]
    w_ = mw[mp_macro]
    h_ = mh[mp_macro]
    offx = np.where(s < w_, s - w_ / 2, np.where(s < w_ + h_, w_ / 2,
           np.where(s < 2 * w_ + h_, w_ / 2 - (s - w_ - h_), -w_ / 2)))
    offy = np.where(s < w_, -h_ / 2, np.where(s < w_ + h_, -h_ / 2 + (s - w_),
           np.where(s < 2 * w_ + h_, h_ / 2, h_ / 2 - (s - 2 * w_ - h_))))
    offx = np.round(offx * 2) / 2
    offy = np.round(offy * 2) / 2
    mp_net = nets_near(mpos[mp_macro, 0] + offx, mpos[mp_macro, 1] + offy)
    io_net = nets_near(iopos[:, 0], iopos[:, 1])

    # pre-permutation ids: std 0..n_std-1, macros n_std.., io after
    perm = rng.permutation(n_inst)            # new id of old instance k
    net_of_std_pin = np.concatenate([np.repeat(g, p.shape[1]) for g, p in groups])
    std_pin_node = np.concatenate([p.ravel() for _, p in groups])
    all_net = np.concatenate([net_of_std_pin, mp_net, io_net])
    all_node = np.concatenate([std_pin_node, n_std + mp_macro, n_std + n_mac + np.arange(n_io)])
    all_off = np.concatenate([np.zeros((std_pin_node.size, 2)),
                              np.stack([offx, offy], axis=1),
                              np.zeros((n_io, 2))])
    o = np.argsort(all_net, kind="stable")
    all_net, all_node, all_off = all_net[o], all_node[o], all_off[o]
    counts = np.bincount(all_net, minlength=n_nets)
    net_ptr = np.zeros(n_nets + 1, dtype=np.int64)
    np.cumsum(counts, out=net_ptr[1:])

    flags_old = np.zeros(n_inst, dtype=np.uint8)
    flags_old[n_std:n_std + n_mac] = MACRO | (0 if cfg.movable_macros else FIXED)
    flags_old[n_std + n_mac:] = FIXED
    size_old = np.zeros((n_inst, 2))
    size_old[:n_std, 0] = std_w
    size_old[:n_std, 1] = 1.0
    size_old[n_std:n_std + n_mac] = msz
    fixed_pos_old = np.zeros((n_inst, 2))
    fixed_pos_old[n_std:n_std + n_mac] = mpos
    fixed_pos_old[n_std + n_mac:] = iopos

    inv = np.empty(n_inst, dtype=np.int64)
    inv[perm] = np.arange(n_inst)
    node_flags = flags_old[inv]
    node_size = size_old[inv].astype(np.float32)
    fixed_pos = fixed_pos_old[inv]
    pin_node = perm[all_node]

    # initial signal: a centre-concentrated warp of the hidden lattice (normal
    # quantiles, sd = die side / 6) plus independent noise per column pair
    from scipy.special import ndtri
    ncols = cfg.ncols
    g0_old = np.zeros((n_inst, ncols), dtype=np.float64)
    kx = np.arange(n_std) % lat_w
    ky = np.arange(n_std) // lat_w
    sd = die_side / 6.0
    wx = sd * ndtri((kx + 0.5) / lat_w)
    wy = sd * ndtri((ky + 0.5) / lat_h)
    jitter = die_side / max(lat_w, 1)
    for c in range(ncols // 2):
        g0_old[:n_std, 2 * c] = np.clip(wx + rng.normal(0.0, jitter, n_std), -half, half)
        g0_old[:n_std, 2 * c + 1] = np.clip(wy + rng.normal(0.0, jitter, n_std), -half, half)
        g0_old[n_std:, 2 * c] = fixed_pos_old[n_std:, 0]
        g0_old[n_std:, 2 * c + 1] = fixed_pos_old[n_std:, 1]
    g0 = g0_old[inv]

    return dict(
        name=cfg.name,
        n_inst=n_inst,
        node_flags=node_flags,
        node_size=node_size,
        net_ptr=net_ptr.astype(np.int32),
        pin_node=pin_node.astype(np.int32),
        pin_off=all_off.astype(np.float32),
        die=die,
        g0=g0.astype(np.float32),
    )


def summary(nl: dict) -> dict:
    deg = np.diff(nl["net_ptr"])
    f = nl["node_flags"]
    return dict(name=nl["name"], n_inst=int(nl["n_inst"]), n_nets=int(deg.size),
                n_pins=int(nl["pin_node"].size), max_deg=int(deg.max()),
                n_fixed=int(((f & FIXED) != 0).sum()), n_macro=int(((f & MACRO) != 0).sum()),
                die_side=float(nl["die"][2] - nl["die"][0]))


def uniform_signal(nl: dict, ncols: int, seed: int) -> np.ndarray:
    """GSP initialization's starting signal (Section IV, step 1): movable
    instances at independent uniform positions in the die (one draw per
    column), fixed ones at their positions (taken from ``g0``)."""
    rng = np.random.default_rng(seed)
    die = nl["die"].astype(np.float64)
    n = nl["n_inst"]
    G = np.empty((n, ncols), np.float64)
    for c in range(ncols):
        lo, hi = (die[0], die[2]) if c % 2 == 0 else (die[1], die[3])
        G[:, c] = rng.uniform(lo, hi, n)
    fixed = (nl["node_flags"] & FIXED) != 0
    G[fixed] = np.tile(nl["g0"][fixed, :2].astype(np.float64), (1, ncols // 2))
    return G.astype(np.float32)
