"""Benchmark of the end-to-end planning step on one MI355X.

One step = mdp_build of the paper-shaped instance (100x100 cells, 120 layers,
5000 flow realizations, 16 headings, all three missions from one histogram
pass) + mdp_value_iterate to convergence for each mission + mdp_policy for each
mission. Inputs are resident in HBM before the timed region.

Prints one JSON line: whole-step throughput in build samples per second, the
build and value-iteration rates on their own, a roofline entry per hot kernel
(live HIP-event launch durations) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X figures (public datasheet): 256 CUs at 2.4 GHz, 4 SIMD x 16 lanes each
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9   # one VALU lane-op per lane per clock: 3.93e13 /s
FP32_VECTOR = 157.3e12                 # packed-FMA FP32 vector peak (FLOP/s)
HBM_BW = 8.0e12                        # bytes/s


def cpu_baseline(w, seconds: float = 12.0):
    """The CPU oracle on a bounded random sample of rows of the same workload
    (one core, as the paper's sequential baseline)."""
    import numpy as np

    import oracle

    rng = np.random.default_rng(123)
    p = w.problem
    nc, na, nr = p["nx"] * p["ny"], w.n_actions, p["n_real"]
    n_rows = n_samples = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        t = int(rng.integers(0, p["nt"]))
        c = int(rng.integers(0, nc))
        a = int(rng.integers(0, na))
        oracle.row(w, t, c, a)
        n_rows += 1
        n_samples += nr
    dt = time.perf_counter() - t0
    return dict(value=n_samples / dt, unit="samples/s", cores=1, kind="oracle",
                sample=f"{n_rows} random (t, cell, action) rows of the same workload, "
                       f"{n_samples} realization landings, full-domain binning and fp64 rewards, "
                       f"{dt:.1f} s on one host core")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--near-edge", action="store_true", help="also count near-edge samples")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the planner has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2109_00857_amd import mdp, workloads as W

    w = W.config2()
    p = dict(w.problem)
    if args.near_edge:
        p["flags"] |= mdp.MDP_FLAG_NEAR_EDGE
    missions = w.missions()
    pl = mdp.Planner(0)
    env = pl.upload_env(w)
    sizes = mdp.mdp_build_query(p)
    model, st0 = pl.build(p, env)  # sizes the model (untimed)
    assert st0["status"] == mdp.MDP_OK, st0
    nnz = st0["nnz"]
    model = pl.alloc_model(p, nnz)
    scratch = pl.scratch(p)
    ns = sizes["n_states"]
    vs = [torch.zeros(ns, dtype=torch.float64, device=pl.device) for _ in missions]
    pis = [torch.empty(ns, dtype=torch.int32, device=pl.device) for _ in missions]
    bstat = mdp.stats_buffer(mdp.MdpBuildStats)
    vstats = [mdp.stats_buffer(mdp.MdpViStats) for _ in missions]
    stream = torch.cuda.current_stream()

    def step():
        mdp.mdp_build(pl.ctx, p, env, model, scratch, bstat, stream)
        for k, m in enumerate(missions):
            vs[k].zero_()
            mdp.mdp_value_iterate(pl.ctx, p, model, m, 1e-6, 100000, vs[k], scratch, vstats[k], stream)
            mdp.mdp_policy(pl.ctx, p, model, m, vs[k], pis[k], stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    mdp.mdp_ctx_profile(pl.ctx, True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    mdp.mdp_ctx_profile(pl.ctx, False)
    ms_step = ev0.elapsed_time(ev1) / args.steps
    bs = mdp.read_stats(bstat, mdp.MdpBuildStats)
    vst = [mdp.read_stats(b, mdp.MdpViStats) for b in vstats]
    assert bs["status"] == mdp.MDP_OK and all(v["status"] == mdp.MDP_OK for v in vst), (bs, vst)

    kt = {k: mdp.mdp_ctx_profile_read(pl.ctx, k) for k in
          (mdp.MDP_KERNEL_BUILD, mdp.MDP_KERNEL_VI_SWEEP, mdp.MDP_KERNEL_POLICY, mdp.MDP_KERNEL_COPY)}
    n_b, ms_b = kt[mdp.MDP_KERNEL_BUILD]
    n_v, ms_v = kt[mdp.MDP_KERNEL_VI_SWEEP]
    nominal = w.nominal_samples
    K, na = p["n_modes"], w.n_actions
    rows, nst = sizes["n_rows"], sizes["n_states"]

    # Build kernel: algorithmic VALU lane-ops per sample = X, Y adds and the two
    # floor conversions of cell() (4), plus the 2K + 2 FMAs of velocity synthesis
    # and position per (layer, cell, realization) shared by the N_a actions.
    ops_per_sample = 4.0 + (2.0 * K + 2.0) / na
    builds = n_b // max(1, bs["n_slabs"])
    build_ops = ops_per_sample * nominal
    build_s = ms_b / 1e3 / builds           # all passes of one build
    build_launch_s = ms_b / 1e3 / n_b       # one launch
    ach_alu = build_ops / bs["n_slabs"] / build_launch_s
    # VI sweep: compulsory bytes of the stored format per sweep.
    sweep_bytes = 8 * (rows + 1) + 4 * rows + 6 * nnz + 8 * nst + 8 * nst
    sweep_s = ms_v / 1e3 / n_v
    ach_hbm = sweep_bytes / sweep_s
    sweeps_per_step = sum(v["sweeps"] for v in vst)

    roof_build = dict(bound="alu", achieved=ach_alu / 1e12, peak=VALU_LANE_OPS / 1e12, unit="Top/s",
                      frac=ach_alu / VALU_LANE_OPS, traffic=None,
                      kernel="k_build", ops_per_sample=ops_per_sample,
                      launch_ms=build_launch_s * 1e3, fp32_flops_frac=None)
    # FP32 arithmetic share: 2 adds + (2K+2) FMAs (2 flops) per N_a samples
    flops = (2.0 + 2.0 * (2.0 * K + 2.0) / na) * nominal / bs["n_slabs"]
    roof_build["fp32_flops_frac"] = flops / build_launch_s / FP32_VECTOR
    roof_vi = dict(bound="hbm", achieved=ach_hbm / 1e9, peak=HBM_BW / 1e9, unit="GB/s",
                   frac=ach_hbm / HBM_BW, traffic=None, kernel="k_vi_sweep",
                   bytes_per_sweep=sweep_bytes, launch_ms=sweep_s * 1e3)
    dominant = roof_build if ms_b >= ms_v else roof_vi

    out = {
        "metric": "MDP build samples/s + VI sweeps/s (% roofline); p50/p99 plan latency served",
        "value": nominal / (ms_step / 1e3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 landings, f64 values",
        "data": "synthetic",
        "config": {"workload": "paper-shaped single instance: 100x100 cells, 120 layers, 10 modes, "
                               "5000 AR(1) realizations, 16 headings, 5x5 sub-grid, 4 moving discs, "
                               "time + energy + net-energy missions",
                   "rows": rows, "nnz": nnz, "samples_per_step": nominal,
                   "near_edge_counted": bool(args.near_edge)},
        "build_samples_per_s": nominal / build_s,
        "build_ms": build_s * 1e3,
        "vi_sweeps_per_s": 1e3 / (ms_v / n_v),
        "vi_sweeps_per_step": sweeps_per_step,
        "vi_ms_per_step": ms_v / args.steps,
        "policy_ms_per_step": kt[mdp.MDP_KERNEL_POLICY][1] / args.steps,
        "copy_ms_per_step": kt[mdp.MDP_KERNEL_COPY][1] / args.steps,
        "roofline": dominant,
        "rooflines": {"build": roof_build, "vi_sweep": roof_vi},
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(w)
        out["cpu_baseline"] = cb
        out["speedup_vs_oracle_1core"] = out["build_samples_per_s"] / cb["value"]
    pl.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
