#!/usr/bin/env python3
"""Benchmark of the area-hint refinement initializer on one MI355X.

One step = the whole hot path on the 2.2M-cell workload: the netlist graph
build (macro pin expansion, clique/star expansion, canonical CSR), then
Algorithm 1 with T_hint = 3 rounds (area hints, absolute-degree
normalisation and Gershgorin lambda_up, the order-8 three-band filter on 4
float32 columns, relaxation), then the HPWL score.  Inputs are seeded,
synthetic and resident in HBM before timing starts.

Prints one JSON line.  The roofline entry is for the dominant kernel (the
SpMM hop): algorithmic bytes per launch over its average duration, measured
with HIP events recorded on the stream the hops run on.  The line also holds
the plain filter and its learned surrogate side by side on the same graph
(device time per call, hop traffic, relative error, HPWL).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MODEL = os.path.join(ROOT, "paper_2511_10073_amd", "weights", "surrogate_bank248.json")
# The hop kernels and the execution layout whose gathers they serve.
HOP_SRCS = [os.path.join(ROOT, "paper_2511_10073_amd", "csrc", f) for f in ("filter.hip", "layout.hip")]

# HBM bytes per k_hop launch on large-2.2M from two rocprofv3 counter passes
# (FETCH_SIZE, WRITE_SIZE) scaled by the same counters for a 1 GiB device
# copy; valid only for the hop and layout sources they were taken with.
HOP_TRAFFIC = {"workload": "large-2.2M",
               "sources_sha256": "646d488cda3753083e8519ebe50109b5c8bb9f8acb4cd2a65d4739fd09c61e49",
               "bytes_per_launch": 1419239714,
               "source": "profiles/k_hop_large-2.2M_hbm_traffic.md"}


def hop_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for p in HOP_SRCS:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def hop_traffic(workload):
    if workload != HOP_TRAFFIC["workload"] or hop_sources_sha() != HOP_TRAFFIC["sources_sha256"]:
        return None
    return HOP_TRAFFIC["bytes_per_launch"]


WORKLOADS = {
    # name: (netlist config attribute, bins, filter bank)
    "large-2.2M": ("LARGE", 32),
    "mid-210k": ("MID", 32),
    "tiny-2k": ("TINY", 8),
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large-2.2M", choices=sorted(WORKLOADS))
    ap.add_argument("--rounds", type=int, default=3, help="T_hint")
    ap.add_argument("--gamma", type=float, default=0.5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-plain comparison")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched 64-netlist filter")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (counter calibration)")
    return ap.parse_args()


def calibrate_copy(mib):
    """A plain copy kernel of known size, for scaling memory counters."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.arange(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read": n * 4, "bytes_written": n * 4, "launches": 3}))


def cpu_baseline(nl, bins, spec_o, rounds):
    """The FP64 oracle on a bounded sample of the same workload: one
    refinement round (graph build + order-8 bank filter) and the HPWL,
    extrapolated to the T_hint rounds of one initializer call."""
    from oracle import ahr_oracle as O
    p = O.HintParams(nbx=bins, nby=bins)
    t0 = time.perf_counter()
    g = O.build_graph(nl, p, nl["g0"][:, :2])
    t1 = time.perf_counter()
    out = O.apply_filter(nl, g, spec_o, nl["g0"])
    t2 = time.perf_counter()
    O.hpwl(nl, out)
    t3 = time.perf_counter()
    ms = 1e3 * (rounds * (t2 - t0) + (t3 - t2))
    return {"value": round(ms, 1), "unit": "ms", "cores": 1, "kind": "oracle",
            "sample": (f"one refinement round (graph build {t1 - t0:.1f} s + order-8 bank filter "
                       f"{t2 - t1:.1f} s) and HPWL ({t3 - t2:.1f} s) of the same workload, "
                       f"round extrapolated to T_hint={rounds}; numpy/scipy, single thread")}


def learned_vs_plain(A, torch, np, nl, net, params, spec, g0, reps):
    """The plain order-8 bank filter and its learned surrogate on the graph
    of the initial placement: device time of one filter call each (HIP
    events on the launch stream, mean of `reps` calls), the bytes their hops
    move, the learned output's centred relative error against the plain one
    over the movable instance rows, and the HPWL of both outputs."""
    if not os.path.exists(MODEL):
        return {"error": f"no trained model at {os.path.relpath(MODEL, ROOT)}"}
    model = A.Mlp.load(MODEL)
    gr = A.Graph(net, params, g0)
    y = torch.empty_like(g0)
    yl = torch.empty_like(g0)
    fb = []

    def plain():
        gr.filter(spec, g0, out=y)

    def learned():
        fb.append(gr.filter_learned(spec, model, g0, out=yl)[1])

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        A.profile_read(reset=True)
        A.profile_enable(True)
        fn()
        torch.cuda.synchronize()
        A.profile_enable(False)
        prof = A.profile_read(reset=True)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(reps):
            fn()
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / reps
        return {"ms": round(ms, 4), "hop_launches": prof["hop_launches"], "hop_bytes": int(prof["hop_bytes"]),
                "hop_gbs": round(prof["hop_bytes"] / (ms * 1e-3) / 1e9, 1), "mlp_ms": round(prof["mlp_ms"], 4)}

    tp = timed(plain)
    tl = timed(learned)
    h_p = gr.hpwl(y).cpu().numpy()
    h_l = gr.hpwl(yl).cpu().numpy()
    gr.close()
    mov = np.flatnonzero((nl["node_flags"][:int(nl["n_inst"])] & 1) == 0)
    a = yl.cpu().numpy().astype(np.float64)[mov]
    b = y.cpu().numpy().astype(np.float64)[mov]
    rel = float(np.linalg.norm(a - b) / np.linalg.norm(b - b.mean(axis=0)))
    return {"plain": tp, "learned": tl, "speedup": round(tp["ms"] / tl["ms"], 3), "rel_err": rel,
            "hpwl_plain": [float(v) for v in h_p], "hpwl_learned": [float(v) for v in h_l],
            "hpwl_delta": float(np.max(np.abs(h_l - h_p) / h_p)), "used_fallback": bool(fb[-1]),
            "model": {"file": os.path.relpath(MODEL, ROOT), "validated": model.validated,
                      "heldout_rel_err_mean": model.summary.get("rel_err_mean")},
            "bounds": {"rel_err": 1e-3, "hpwl_delta": 2e-3}}


def learned_initializer(A, torch, np, nl, net, params, spec, g0, rounds, gamma, steps, plain_ms, plain_out,
                        plain_hpwl):
    """The same initializer step with the learned filter in every round of
    Algorithm 1 (graph build + T_hint rounds + HPWL), timed like the plain
    step, and its final placement and HPWL against the plain step's."""
    if not os.path.exists(MODEL):
        return {"error": f"no trained model at {os.path.relpath(MODEL, ROOT)}"}
    model = A.Mlp.load(MODEL)
    out = torch.empty_like(g0)
    hp = torch.empty_like(plain_hpwl)
    fb = []

    def step():
        gr = A.Graph(net, params, None)
        fb.append(gr.refine_learned(spec, model, g0, rounds, gamma, out=out)[1])
        gr.hpwl(out, out=hp)
        gr.close()

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    mov = np.flatnonzero((nl["node_flags"][:int(nl["n_inst"])] & 1) == 0)
    a = out.cpu().numpy().astype(np.float64)[mov]
    b = plain_out.cpu().numpy().astype(np.float64)[mov]
    h_l, h_p = hp.cpu().numpy(), plain_hpwl.cpu().numpy()
    return {"ms": round(ms, 3), "speedup_vs_plain": round(plain_ms / ms, 3),
            "rel_err_vs_plain": float(np.linalg.norm(a - b) / np.linalg.norm(b - b.mean(axis=0))),
            "hpwl": [float(v) for v in h_l], "hpwl_delta": float(np.max(np.abs(h_l - h_p) / h_p)),
            "used_fallback": bool(fb[-1])}


def batch_bins(n_inst):
    """Bin grid of a batch member: about 200 cells per bin, 8x8 to 32x32."""
    b = int(round((n_inst / 200.0) ** 0.5))
    return min(32, max(8, b))


def batched(A, torch, np, N, spec, reps):
    """The batched workload: 64 netlists of 5k-200k cells (log-uniform,
    2-5 % macros) filtered with the order-8 bank on 4 columns in one
    replayed HIP graph, with the launch shape the tuner picks.  Compared
    with filtering the members one after another (single-graph calls, same
    launch shape); the two outputs must be bit-identical."""
    t0 = time.perf_counter()
    members = N.batch_sizes()
    nls = [N.generate(N.batch_member(*m)) for m in members]
    gen_s = time.perf_counter() - t0
    nets = [A.Netlist(nl) for nl in nls]
    params = [A.hint_params(nbx=batch_bins(nl["n_inst"]), nby=batch_bins(nl["n_inst"])) for nl in nls]
    pos = torch.as_tensor(np.concatenate([nl["g0"] for nl in nls])).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = A.Batch(nets, params, pos)
    build_s = time.perf_counter() - t0
    lanes, ct, tune_ms = b.autotune(spec, pos.shape[1])
    out = torch.empty_like(pos)
    # algorithmic hop bytes of one call (direct launch, profiled)
    b.filter(spec, pos, out=out, use_graph=False)
    torch.cuda.synchronize()
    A.profile_read(reset=True)
    A.profile_enable(True)
    b.filter(spec, pos, out=out, use_graph=False)
    torch.cuda.synchronize()
    A.profile_enable(False)
    prof = A.profile_read(reset=True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for _ in range(2):
        b.filter(spec, pos, out=out)
    ev[0].record()
    for _ in range(reps):
        b.filter(spec, pos, out=out)
    ev[1].record()
    # the same work one member at a time
    saved = A.filter_get_tune()
    A.filter_tune(lanes, -1)
    graphs = [A.Graph(net, p, pos[lo:hi]) for net, p, lo, hi in zip(nets, params, b.offsets[:-1], b.offsets[1:])]
    xs = [pos[lo:hi].contiguous() for lo, hi in zip(b.offsets[:-1], b.offsets[1:])]
    ys = [torch.empty_like(x) for x in xs]
    for g, x, y in zip(graphs, xs, ys):
        g.filter(spec, x, out=y)
    ev[2].record()
    for _ in range(reps):
        for g, x, y in zip(graphs, xs, ys):
            g.filter(spec, x, out=y)
    ev[3].record()
    torch.cuda.synchronize()
    same = bool(torch.equal(out, torch.cat(ys)))
    A.filter_tune(*saved)
    for g in graphs:
        g.close()
    inf = b.info()
    b.close()
    ms = ev[0].elapsed_time(ev[1]) / reps
    seq_ms = ev[2].elapsed_time(ev[3]) / reps
    return {"n_graphs": inf["n_graphs"], "n_inst": inf["n_inst"], "n_tot": inf["n_tot"],
            "nnz": inf["nnz_net"] + inf["nnz_hint"], "cells_min": int(min(nl["n_inst"] for nl in nls)),
            "cells_max": int(max(nl["n_inst"] for nl in nls)), "ncols": int(pos.shape[1]),
            "tuned": {"lanes_per_row": lanes, "col_tile": ct, "ms": round(tune_ms, 4)},
            "ms": round(ms, 4), "hop_bytes": int(prof["hop_bytes"]),
            "gbs": round(prof["hop_bytes"] / (ms * 1e-3) / 1e9, 1),
            "members_one_by_one_ms": round(seq_ms, 4), "speedup": round(seq_ms / ms, 3),
            "bit_identical_to_members": same, "build_s": round(build_s, 2), "generator_s": round(gen_s, 1)}


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (multi-GPU sharding is "
                                   "design-only, see the design notes)"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2511_10073_amd as A
    from synth import netlist as N

    cfg_name, bins = WORKLOADS[args.workload]
    cfg = getattr(N, cfg_name)
    t = time.perf_counter()
    nl = N.generate(cfg)
    gen_s = time.perf_counter() - t
    ncols = nl["g0"].shape[1]
    dev = torch.device("cuda:0")
    net = A.Netlist(nl, dev)
    g0 = torch.as_tensor(nl["g0"]).to(dev)
    params = A.hint_params(nbx=bins, nby=bins)
    ks, alphas = (2, 4, 8), (0.2, 0.3, 0.5)
    spec = A.filter_spec(ks, alphas)
    out = torch.empty_like(g0)
    hp = torch.empty(ncols // 2, dtype=torch.float64, device=dev)

    def step():
        gr = A.Graph(net, params, None)
        gr.refine(spec, g0, args.rounds, args.gamma, out=out)
        gr.hpwl(out, out=hp)
        gr.close()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed steps: events around the hop launches only (the roofline's kernel)
    A.profile_read(reset=True)
    A.profile_enable(True, hops_only=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    A.profile_enable(False)
    prof = A.profile_read(reset=True)
    ms = 1e3 * (t1 - t0) / args.steps
    # stage breakdown from further steps with every stage timed (outside the
    # timed region: the stage events add about 0.3 ms per step)
    stage_steps = min(args.steps, 3)
    A.profile_enable(True)
    for _ in range(stage_steps):
        step()
    torch.cuda.synchronize()
    A.profile_enable(False)
    sprof = A.profile_read(reset=True)

    # graph sizes of the last round (for the record)
    gr = A.Graph(net, params, g0)
    info = gr.info()
    gr.close()

    hop_avg_ms = prof["hop_ms"] / max(prof["hop_launches"], 1)
    hop_bytes = prof["hop_bytes"] / max(prof["hop_launches"], 1)
    achieved = hop_bytes / (hop_avg_ms * 1e-3) / 1e9
    per_step = {k: round(sprof[k] / stage_steps, 3) for k in
                ("build_ms", "hints_ms", "norm_ms", "expand_ms", "hop_ms", "relax_ms", "hpwl_ms")}
    filt_ms = per_step["expand_ms"] + per_step["hop_ms"]
    rec = {
        "metric": "initializer ms & GB/s at 2.2M cells; learned vs plain at <=1e-3 rel err",
        "value": round(ms, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload} area-hint refinement initializer (graph build + T_hint="
                               f"{args.rounds} rounds of hints + order-8 bank filter on {ncols} columns + "
                               f"relax, then HPWL)",
                   "n_inst": int(nl["n_inst"]), "n_nets": int(nl["net_ptr"].size - 1),
                   "n_pins": int(nl["pin_node"].size), "n_tot": info["n_tot"], "nnz_net": info["nnz_net"],
                   "nnz_hint": info["nnz_hint"], "bins": f"{bins}x{bins}", "bank": {"k": ks, "alpha": alphas},
                   "ncols": ncols, "T_hint": args.rounds, "gamma": args.gamma},
        "roofline": {"bound": "hbm", "kernel": "k_hop (SpMM hop)", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": hop_traffic(args.workload), "avg_launch_us": round(hop_avg_ms * 1e3, 2),
                     "algorithmic_bytes_per_launch": int(hop_bytes), "launches": prof["hop_launches"]},
        "stages_ms_per_step": per_step,
        "stages_note": f"from {stage_steps} further steps with every stage timed (the timed steps time the hop only)",
        "filter_phase_gbs": round(prof["hop_bytes"] / args.steps / (filt_ms * 1e-3) / 1e9, 1) if filt_ms else None,
        "hpwl": [float(v) for v in hp.cpu().numpy()],
        "generator_s": round(gen_s, 1),
    }
    if not args.no_learned:
        rec["learned_vs_plain"] = learned_vs_plain(A, torch, np, nl, net, params, spec, g0, reps=10)
        rec["learned_initializer"] = learned_initializer(A, torch, np, nl, net, params, spec, g0, args.rounds,
                                                         args.gamma, args.steps, ms, out, hp)
    if not args.no_batched:
        rec["batched"] = batched(A, torch, np, N, spec, reps=10)
    if not args.no_cpu_baseline:
        from oracle import ahr_oracle as O
        rec["cpu_baseline"] = cpu_baseline(nl, bins, O.FilterSpec(ks=ks, alphas=alphas), args.rounds)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
