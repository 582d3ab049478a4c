"""Training of the learned filter surrogate on the device.

Every numeric step runs in libahr: the plain filter (targets), the
features and hops, the float32 forward/backward, Adam.  The host only fits
the four linear weights beta of h0..h3 (a 4x4 least-squares system) and
drives the loop.

The training set spans netlist sizes, so that the scale-free features and
the log(s_c / r_c) feature see the sizes the filter is served at:
`--train` netlists of the mid-210k shape plus `--train-sized` netlists whose
sizes are log-uniform between 300k and 2.2M cells (`synth.netlist.sized`).
Held out: `--heldout` mid-210k netlists and `--heldout-large` netlists of the
large-2.2M shape, reported separately.

    python -m paper_2511_10073_amd.train --train 160 --train-sized 40 --heldout 16 --heldout-large 4

The result is written as JSON (parameters, beta, the validation flag and a
summary of the held-out evaluation) and read back with `Mlp.load`.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import time

import numpy as np
import torch

from . import (MLP_NPARAM, Graph, Mlp, Netlist, filter_spec, hint_params, mlp_adam, mlp_loss_grad)

HIDDEN = 64
FEAT_PAD = 8
NFEAT = 7
NHOPS = 4       # h0 (the input) .. h3
DEFAULT_MODEL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "surrogate_bank248.json")
W3_OFF = HIDDEN * FEAT_PAD + HIDDEN + HIDDEN * HIDDEN + HIDDEN
B3_OFF = W3_OFF + HIDDEN


def init_params(seed: int) -> torch.Tensor:
    """He-style hidden layers; a zero output layer, so the untrained model is
    exactly the linear combination of the hops."""
    g = torch.Generator().manual_seed(seed)
    p = torch.zeros(MLP_NPARAM)
    w1 = torch.randn(HIDDEN, NFEAT, generator=g) * math.sqrt(2.0 / NFEAT)
    W1 = torch.zeros(HIDDEN, FEAT_PAD)
    W1[:, :NFEAT] = w1
    p[:HIDDEN * FEAT_PAD] = W1.reshape(-1)
    o2 = HIDDEN * FEAT_PAD + HIDDEN
    p[o2:o2 + HIDDEN * HIDDEN] = (torch.randn(HIDDEN, HIDDEN, generator=g) * math.sqrt(2.0 / HIDDEN)).reshape(-1)
    return p


def collect(nl: dict, params, spec, rows=None, seed=0, device="cuda"):
    """Targets (plain filter), hops, features and column statistics of one
    netlist's initial signal, for its movable rows (or a seeded subset of
    `rows` of them), as host arrays."""
    net = Netlist(nl, device)
    x = torch.as_tensor(nl["g0"]).to(device)
    gr = Graph(net, params, x)
    y = gr.filter(spec, x)
    feats, hops, stats = gr.features(spec, x)
    gr.close()
    mov = np.flatnonzero((nl["node_flags"] & 1) == 0)
    if rows is not None and rows < mov.size:
        mov = np.sort(np.random.default_rng(seed).choice(mov, rows, replace=False))
    C = x.shape[1]
    f = feats.cpu().numpy().reshape(-1, C, FEAT_PAD)[mov]
    return dict(y=y.cpu().numpy()[mov].astype(np.float64), hops=hops.cpu().numpy()[:, mov].astype(np.float64),
                feats=f.reshape(-1, FEAT_PAD), stats=stats.cpu().numpy().astype(np.float64), C=C)


def fit_beta(data: list) -> np.ndarray:
    """Least-squares weights of h0..h3 over the collected rows (4x4 normal
    equations in float64)."""
    G = np.zeros((NHOPS, NHOPS))
    b = np.zeros(NHOPS)
    for d in data:
        H = d["hops"].reshape(NHOPS, -1)
        G += H @ H.T
        b += H @ d["y"].reshape(-1)
    return np.linalg.solve(G, b)


def residual_samples(data: list, beta, device="cuda") -> tuple:
    """Feature rows and residual targets r = (y - sum beta h) / r_c, moved to
    the device once."""
    feats, targets = [], []
    for d in data:
        lin = sum(beta[j] * d["hops"][j] for j in range(NHOPS))
        r = (d["y"] - lin) / d["stats"][2][None, :]
        feats.append(d["feats"])
        targets.append(r.reshape(-1))
    F = torch.as_tensor(np.concatenate(feats).astype(np.float32)).to(device)
    R = torch.as_tensor(np.concatenate(targets).astype(np.float32)).to(device)
    return F, R


def train_mlp(F, R, steps=1000, lr=3e-3, seed=0, log=None):
    """Full-batch Adam on mean (MLP(F) - R)^2 (cosine learning-rate decay).
    Targets are scaled to unit deviation for training; the scale is folded
    back into the linear output layer."""
    sigma = float(np.std(R.cpu().numpy())) or 1.0
    Rn = torch.as_tensor((R.cpu().numpy() / sigma).astype(np.float32)).to(F.device)
    P = init_params(seed).to(F.device)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    t0 = time.time()
    for k in range(1, steps + 1):
        g, loss = mlp_loss_grad(P, F, Rn)
        mlp_adam(P, m, v, g, k, lr * 0.5 * (1 + math.cos(math.pi * k / steps)))
        if log and (k % 100 == 0 or k == 1):
            log(f"step {k} loss {float(loss.cpu()):.4e} ({time.time() - t0:.1f} s)")
    _, loss = mlp_loss_grad(P, F, Rn)
    p = P.cpu().numpy()
    p[W3_OFF:W3_OFF + HIDDEN] *= sigma
    p[B3_OFF] *= sigma
    return torch.as_tensor(p).to(F.device), float(loss.cpu()) * sigma * sigma


def rel_err(y, ref, mov):
    """Centred relative Frobenius error over the given rows (host arrays)."""
    y = np.asarray(y, np.float64)[mov]
    ref = np.asarray(ref, np.float64)[mov]
    return float(np.linalg.norm(y - ref) / np.linalg.norm(ref - ref.mean(axis=0)))


def evaluate(nl: dict, params, spec, model: Mlp, device="cuda"):
    """Relative error and HPWL delta of the learned filter against the plain
    one on a netlist's initial signal (both on the device)."""
    net = Netlist(nl, device)
    x = torch.as_tensor(nl["g0"]).to(device)
    gr = Graph(net, params, x)
    y = gr.filter(spec, x)
    out, fb = gr.filter_learned(spec, model, x)
    lin, _ = gr.filter_learned(spec, Mlp(torch.zeros_like(model.params), model.beta, True), x)
    h_ref = gr.hpwl(y).cpu().numpy()
    h_out = gr.hpwl(out).cpu().numpy()
    gr.close()
    mov = (nl["node_flags"] & 1) == 0
    y, out, lin = y.cpu().numpy(), out.cpu().numpy(), lin.cpu().numpy()
    return dict(rel_err=rel_err(out, y, mov), rel_err_linear=rel_err(lin, y, mov),
                hpwl_delta=float(np.max(np.abs(h_out - h_ref) / h_ref)), fallback=fb)


def main():
    from synth import netlist as N

    ap = argparse.ArgumentParser(description="train the learned filter surrogate")
    ap.add_argument("--train", type=int, default=160, help="mid-210k training netlists")
    ap.add_argument("--train-sized", type=int, default=40, help="training netlists of 300k-2.2M cells")
    ap.add_argument("--heldout", type=int, default=16, help="mid-210k held-out netlists")
    ap.add_argument("--heldout-large", type=int, default=4, help="large-2.2M held-out netlists")
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--rows", type=int, default=20000, help="movable rows sampled per mid-210k training netlist")
    ap.add_argument("--rows-sized", type=int, default=60000, help="movable rows sampled per sized training netlist")
    ap.add_argument("--tol", type=float, default=1e-3, help="validation bound on the mean held-out error")
    ap.add_argument("--out", default=DEFAULT_MODEL)
    args = ap.parse_args()
    spec = filter_spec((2, 4, 8), (0.2, 0.3, 0.5))
    params = hint_params(nbx=32, nby=32)
    t0 = time.time()
    data = []
    for s in range(4000, 4000 + args.train):
        data.append(collect(N.generate(N.sized(N.MID.n_std, s)), params, spec, rows=args.rows, seed=s))
        print(f"collected mid {s} ({time.time() - t0:.0f} s)", flush=True)
    rng = np.random.default_rng(4600)
    sizes = np.exp(rng.uniform(math.log(300_000), math.log(N.LARGE.n_std), args.train_sized)).astype(int)
    for k, n in enumerate(sizes):
        s = 4600 + k
        data.append(collect(N.generate(N.sized(int(n), s)), params, spec, rows=args.rows_sized, seed=s))
        print(f"collected sized {s} ({n} cells, {time.time() - t0:.0f} s)", flush=True)
    beta = fit_beta(data)
    F, R = residual_samples(data, beta)
    del data
    P, loss = train_mlp(F, R, args.steps, args.lr, log=lambda m: print(m, flush=True))
    del F, R
    model = Mlp(P, beta, True)
    res = {"mid": [], "large": []}
    for s in range(4200, 4200 + args.heldout):
        res["mid"].append(evaluate(N.generate(N.sized(N.MID.n_std, s)), params, spec, model))
        print("mid", json.dumps(res["mid"][-1]), flush=True)
    for s in range(4700, 4700 + args.heldout_large):
        cfg = dataclasses.replace(N.LARGE, name=f"large-{s}", seed=s)
        res["large"].append(evaluate(N.generate(cfg), params, spec, model))
        print("large", json.dumps(res["large"][-1]), flush=True)
    summary = dict(train=args.train, train_sized=args.train_sized, sized_cells=[int(v) for v in sizes],
                   heldout=args.heldout, heldout_large=args.heldout_large, steps=args.steps, loss=loss,
                   beta=list(map(float, beta)), tol=args.tol)
    ok = True
    for k, rs in res.items():
        if not rs:
            continue
        e = np.array([r["rel_err"] for r in rs])
        el = np.array([r["rel_err_linear"] for r in rs])
        hd = np.array([r["hpwl_delta"] for r in rs])
        summary[k] = dict(rel_err_mean=float(e.mean()), rel_err_max=float(e.max()),
                          rel_err_linear_mean=float(el.mean()), gain=float(el.mean() - e.mean()),
                          hpwl_delta_max=float(hd.max()))
        ok = ok and bool(e.mean() <= args.tol and hd.max() <= 2e-3)
    summary["validated"] = ok
    save_model(args.out, P, beta, ok, summary)
    print(json.dumps(summary), flush=True)


def save_model(path, P, beta, validated, summary):
    """Write a model as JSON: float32 parameters (exact decimal round trip),
    beta, the validation flag and the training summary."""
    p = P.cpu().numpy().astype(np.float32)
    doc = dict(format="ahr-mlp-2", hidden=HIDDEN, feat_pad=FEAT_PAD, nparam=int(p.size),
               params=[float(v) for v in p], beta=[float(np.float32(b)) for b in beta], validated=bool(validated),
               summary=summary)
    with open(path, "w") as f:
        json.dump(doc, f)


if __name__ == "__main__":
    main()
