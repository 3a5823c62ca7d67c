"""Benchmark of the end-to-end planning step on one MI355X.

One step = mdp_build of the paper-shaped instance (100x100 cells, 120 layers,
5000 flow realizations, 16 headings, all three missions from one histogram
pass) + value iteration to convergence for each mission (the three missions in
one mdp_value_iterate_missions solve, which reads the shared transition entries
once per sweep) + mdp_policy for each mission. Inputs are resident in HBM before
the timed region.

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


# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE on this workload
# (profiles/paper_shaped_step_hbm_counters.md; FETCH_SIZE scaled x2.000 and
# WRITE_SIZE x1.000 by a plain 1 GiB copy). They hold for the kernel source
# whose sha256 prefix is given; after any change the traffic is reported null.
MEASURED_TRAFFIC = {
    "k_vi_sweep_missions<3>": dict(read=416382836, write=14990361, src="paper_2109_00857_amd/csrc/vi.hip",
                                   sha256="1731d5bb665d1631"),
    "k_build": dict(read=443800111, write=882340240, src="paper_2109_00857_amd/csrc/build.hip",
                    sha256="e21e074de0a0dd60"),
}


def measured_traffic(kernel: str):
    """HBM bytes per launch (read + write) measured for this kernel source, or None."""
    import hashlib

    m = MEASURED_TRAFFIC[kernel]
    with open(os.path.join(ROOT, m["src"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != m["sha256"]:
            return None
    return m["read"] + m["write"]


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


def _ev_ms(stream, fn, reps: int) -> float:
    """Mean ms of fn() over reps runs, HIP events on `stream` around the runs."""
    import torch

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def batched_leg(pl, n_inst: int = 64, reps: int = 2) -> dict:
    """The uneven 64-instance batch: one persistent build launch + one sweep launch per
    iteration + policies, replayed from a HIP graph, against the same instances solved
    one after another with the plain calls (build, value iteration, policy) on one stream."""
    import torch

    from paper_2109_00857_amd import mdp, workloads as W

    t_gen = time.perf_counter()
    ws = [W.batched_instance(i) for i in range(n_inst)]
    t_gen = time.perf_counter() - t_gen
    missions = [w.missions()[0] for w in ws]
    envs = [pl.upload_env(w) for w in ws]
    for w, env in zip(ws, envs):  # sub-grid sized from the synthesised velocities (untimed)
        w.problem["sub_hx"], w.problem["sub_hy"] = mdp.mdp_subgrid_auto(pl.ctx, w.problem, env)
    samples = sum(w.nominal_samples for w in ws)
    b = mdp.Batch(pl, [w.problem for w in ws], envs, missions)
    bs = b.build_checked()
    assert all(x["status"] == mdp.MDP_OK for x in bs), bs
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.capture(stream=s)
    s.synchronize()
    b.replay(stream=s)  # warm
    ms_batch = _ev_ms(s, lambda: b.replay(stream=s), reps)
    bst, vst = b.stats()
    assert all(x["status"] == mdp.MDP_OK for x in bst) and all(x["status"] == mdp.MDP_OK for x in vst)
    nnz = [x["nnz"] for x in bst]
    pi_batch = [t.clone() for t in b.pi]
    b.close()
    del b

    # the same instances through the plain single-problem calls, back to back
    models = [pl.alloc_model(w.problem, c) for w, c in zip(ws, nnz)]
    scratch = torch.empty(max(mdp.mdp_build_query(w.problem)["scratch_bytes"] for w in ws), dtype=torch.uint8,
                          device=pl.device)
    vs = [torch.zeros(w.n_states, dtype=torch.float64, device=pl.device) for w in ws]
    pis = [torch.empty(w.n_states, dtype=torch.int32, device=pl.device) for w in ws]
    bstat = [mdp.stats_buffer(mdp.MdpBuildStats) for _ in ws]
    vstat = [mdp.stats_buffer(mdp.MdpViStats) for _ in ws]

    def plain_all():
        for k, w in enumerate(ws):
            mdp.mdp_build(pl.ctx, w.problem, envs[k], models[k], scratch, bstat[k], s)
            vs[k].zero_()
            mdp.mdp_value_iterate(pl.ctx, w.problem, models[k], missions[k], 1e-6, 100000, vs[k], scratch,
                                  vstat[k], s)
            mdp.mdp_policy(pl.ctx, w.problem, models[k], missions[k], vs[k], pis[k], s)

    with torch.cuda.stream(s):
        plain_all()  # warm
        ms_plain = _ev_ms(s, plain_all, reps)
    same = all(torch.equal(a, c) for a, c in zip(pis, pi_batch))
    rows = sum(w.n_rows for w in ws)
    out = dict(instances=n_inst, samples=samples, rows=rows, nnz=sum(nnz), generator_s=t_gen,
               ms_batched_graph=ms_batch, ms_plain_sequential=ms_plain,
               samples_per_s_batched=samples / (ms_batch / 1e3), samples_per_s_plain=samples / (ms_plain / 1e3),
               speedup=ms_plain / ms_batch, policies_equal=bool(same),
               sweeps_max=max(x["sweeps"] for x in vst))
    del models, scratch, vs, pis
    torch.cuda.empty_cache()
    return out


def _served_trace(seconds: float, rate: float, seed: int = 7):
    """Poisson arrivals; 90 % uneven batched-mix requests, 10 % paper-shaped ones, each
    request's seed 100000 + j and its mission uniform over the three."""
    import numpy as np

    from paper_2109_00857_amd import workloads as W

    rng = np.random.default_rng(seed)
    t, arr = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            break
        arr.append(t)
    reqs = []
    for j in range(len(arr)):
        if rng.random() < 0.1:
            m = int(rng.integers(0, 3))
            w = W.config2(seed=100000 + j, missions=(m,))
            if m != W.MISSION_NET_ENERGY:
                w.gbar = None
        else:
            w = W.batched_instance(j, base_seed=100000)
            m = w.missions()[0]
        reqs.append((w, m))
    return arr, reqs


def served_inputs(pl, seconds: float, rate: float):
    """The trace's requests with their environments resident on the device and
    their sub-grids sized (outside any timed region)."""
    from paper_2109_00857_amd import mdp

    arr, reqs = _served_trace(seconds, rate)
    envs = [pl.upload_env(w) for w, _ in reqs]
    for (w, _), env in zip(reqs, envs):  # requests arrive with their sub-grid sized
        if w.problem["sub_hx"] == 0 and w.problem["sub_hy"] == 0:
            w.problem["sub_hx"], w.problem["sub_hy"] = mdp.mdp_subgrid_auto(pl.ctx, w.problem, env)
    return arr, reqs, envs


def served_leg(pl, seconds: float, rate: float, pool_gib: float = 48.0, build_share: int = 100,
               sweeps_per_step: int = 32, sequential: bool = True, trace=None) -> dict:
    """The served trace through the continuous-batching server, then the same trace
    through sequential plain solves (first come, first served, one at a time)."""
    import numpy as np
    import torch

    from paper_2109_00857_amd import mdp

    t_gen = time.perf_counter()
    if trace is None:
        trace = served_inputs(pl, seconds, rate)
    arr, reqs, envs = trace
    t_gen = time.perf_counter() - t_gen
    n = len(reqs)
    samples = sum(w.nominal_samples for w, _ in reqs)

    def stats(lat, wall):
        a = np.array([lat[j] for j in range(n)]) * 1e3
        return dict(p50_ms=float(np.percentile(a, 50)), p99_ms=float(np.percentile(a, 99)),
                    mean_ms=float(a.mean()), max_ms=float(a.max()), wall_s=wall,
                    requests_per_s=n / wall, samples_per_s=samples / wall)

    s = torch.cuda.Stream()
    srv = mdp.Server(pl, pool_bytes=int(pool_gib * (1 << 30)), max_inflight=64, sweeps_per_step=sweeps_per_step,
                     stream=s, build_share=build_share)
    # warm the server's code paths on the first two requests (results discarded)
    for j in range(min(2, n)):
        srv.submit(-1 - j, reqs[j][0].problem, envs[j], reqs[j][1])
    while srv.step():
        pass
    srv.poll()
    first_step = srv.info()["steps"]  # step numbers continue after the warm-up
    lat, status, admit = {}, {}, {}
    step_start = {}  # step number -> host time it started
    i, n_steps, t_steps = 0, 0, 0.0
    t0 = time.perf_counter()
    while len(lat) < n:
        now = time.perf_counter() - t0
        while i < n and arr[i] <= now:
            srv.submit(i, reqs[i][0].problem, envs[i], reqs[i][1])
            i += 1
        if i - len(lat) > 0:
            ts = time.perf_counter()
            n_steps += 1
            step_start[n_steps] = ts - t0
            srv.step()
            t_steps += time.perf_counter() - ts
        elif i < n:
            time.sleep(max(0.0, arr[i] - (time.perf_counter() - t0)))
        t = time.perf_counter() - t0
        for rec in srv.poll():
            lat[rec["tag"]] = t - arr[rec["tag"]]
            status[rec["tag"]] = rec["status"]
            admit[rec["tag"]] = step_start.get(rec["admit_step"] - first_step, arr[rec["tag"]]) - arr[rec["tag"]]
    wall_served = time.perf_counter() - t0
    srv.close()
    del srv
    torch.cuda.empty_cache()
    served = stats(lat, wall_served)
    served["all_ok"] = all(v == mdp.MDP_OK for v in status.values())
    served["steps"] = n_steps
    served["mean_step_ms"] = 1e3 * t_steps / max(n_steps, 1)
    served["mean_queue_wait_ms"] = 1e3 * float(np.mean([max(0.0, admit[j]) for j in range(n)]))
    if not sequential:
        return dict(requests=n, samples=samples, served=served, build_share=build_share,
                    sweeps_per_step=sweeps_per_step)

    # sequential plain solves of the same trace
    lat2 = {}
    bst, vst = mdp.stats_buffer(mdp.MdpBuildStats), mdp.stats_buffer(mdp.MdpViStats)
    with torch.cuda.stream(s):
        t0 = time.perf_counter()
        for j, (w, m) in enumerate(reqs):
            now = time.perf_counter() - t0
            if now < arr[j]:
                time.sleep(arr[j] - now)
            p = dict(w.problem, mission_mask=1 << m)
            sz = mdp.mdp_build_query(p)
            model = pl.alloc_model(p, sz["nnz_upper"])
            scratch = pl.scratch(p)
            v = torch.zeros(sz["n_states"], dtype=torch.float64, device=pl.device)
            pi = torch.empty(sz["n_states"], dtype=torch.int32, device=pl.device)
            mdp.mdp_build(pl.ctx, p, envs[j], model, scratch, bst, s)
            mdp.mdp_value_iterate(pl.ctx, p, model, m, 1e-6, 100000, v, scratch, vst, s)
            mdp.mdp_policy(pl.ctx, p, model, m, v, pi, s)
            pi_host = pi.to("cpu", non_blocking=False)
            lat2[j] = time.perf_counter() - t0 - arr[j]
            del model, scratch, v, pi, pi_host
        wall_seq = time.perf_counter() - t0
    torch.cuda.empty_cache()
    seq = stats(lat2, wall_seq)
    return dict(trace=f"Poisson {rate}/s for {seconds} s (seed 7): {n} requests, 90% uneven batched-mix, "
                      f"10% paper-shaped, missions uniform", requests=n, samples=samples, generator_s=t_gen,
                build_share=build_share, sweeps_per_step=sweeps_per_step,
                served=served, sequential_plain=seq,
                p50_speedup=seq["p50_ms"] / served["p50_ms"], p99_speedup=seq["p99_ms"] / served["p99_ms"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--near-edge", action="store_true", help="also count near-edge samples")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-instance batched leg")
    ap.add_argument("--no-served", action="store_true", help="skip the served-trace leg")
    ap.add_argument("--serve-seconds", type=float, default=20.0, help="length of the served trace")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="request arrival rate (per second)")
    ap.add_argument("--build-share", type=int, default=100,
                    help="percent of the GPU's resident workgroups a served build batch may hold")
    ap.add_argument("--serve-sweeps", type=int, default=32, help="most sweeps per served scheduler step")
    ap.add_argument("--no-autotune", action="store_true", help="build with the default launch shape")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch

        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": a.numel() * 4, "copies": 3}))
        return
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
    tune = None
    if not args.no_autotune:  # untimed: pick the build launch shape for this shape class
        tune = mdp.mdp_autotune(pl.ctx, p, env)
    sizes = mdp.mdp_build_query(p)
    model, st0 = pl.build(p, env)  # sizes the model (untimed)
    assert st0["status"] == mdp.MDP_OK, st0
    nnz = st0["nnz"]
    model = pl.alloc_model(p, nnz)
    scratch = pl.scratch(p)
    vi_scratch = torch.empty(len(missions) * sizes["scratch_bytes"], dtype=torch.uint8, device=pl.device)
    ns = sizes["n_states"]
    vs = [torch.zeros(ns, dtype=torch.float64, device=pl.device) for _ in missions]
    pis = [torch.empty(ns, dtype=torch.int32, device=pl.device) for _ in missions]
    bstat = mdp.stats_buffer(mdp.MdpBuildStats)
    vsz = mdp.C.sizeof(mdp.MdpViStats)
    vstat = torch.zeros(len(missions) * vsz, dtype=torch.uint8, pin_memory=True)
    stream = torch.cuda.current_stream()

    def step():
        mdp.mdp_build(pl.ctx, p, env, model, scratch, bstat, stream)
        for v in vs:
            v.zero_()
        mdp.mdp_value_iterate_missions(pl.ctx, p, model, missions, 1e-6, 100000, vs, vi_scratch, vstat, stream)
        for k, m in enumerate(missions):
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
    vst = [mdp.read_stats(vstat[k * vsz:(k + 1) * vsz], mdp.MdpViStats) for k in range(len(missions))]
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
    # VI: compulsory bytes of the stored format for the layers each fused sweep
    # recomputes (sweep k of a solve recomputes layers t < nt - k + 1): per
    # layer 8 B row pointer per row and 6 B per nonzero, read once for all
    # missions, plus per mission still iterating 4 B reward per row and v read
    # and written once per state.
    nt, nc = p["nt"], p["nx"] * p["ny"]
    rp_layer = model["row_ptr"][:: nc * na].cpu().numpy()  # row_ptr at layer starts (+ end)
    nnz_layer = rp_layer[1:] - rp_layer[:-1]
    shared_bytes = 8 * nc * na + 6 * nnz_layer
    mission_bytes = 4 * nc * na + 16 * nc
    solve_bytes = 0
    for k in range(max(v["sweeps"] for v in vst)):
        live = sum(1 for v in vst if v["sweeps"] > k)
        t_hi = max(0, min(nt, nt - k + 1))
        solve_bytes += int(shared_bytes[:t_hi].sum() + live * mission_bytes * t_hi)
    sweep_bytes = int(shared_bytes.sum() + len(missions) * mission_bytes * nt) + 8  # one full fused sweep
    sweep_s = ms_v / 1e3 / n_v
    ach_hbm = solve_bytes * args.steps / (ms_v / 1e3)
    sweeps_per_step = sum(v["sweeps"] for v in vst)

    roof_build = dict(bound="alu", achieved=ach_alu / 1e12, peak=VALU_LANE_OPS / 1e12, unit="Top/s",
                      frac=ach_alu / VALU_LANE_OPS, traffic=measured_traffic("k_build"),
                      kernel="k_build", ops_per_sample=ops_per_sample,
                      launch_ms=build_launch_s * 1e3, fp32_flops_frac=None)
    # FP32 arithmetic share: 2 adds + (2K+2) FMAs (2 flops) per N_a samples
    flops = (2.0 + 2.0 * (2.0 * K + 2.0) / na) * nominal / bs["n_slabs"]
    roof_build["fp32_flops_frac"] = flops / build_launch_s / FP32_VECTOR
    roof_vi = dict(bound="hbm", achieved=ach_hbm / 1e9, peak=HBM_BW / 1e9, unit="GB/s",
                   frac=ach_hbm / HBM_BW, traffic=measured_traffic("k_vi_sweep_missions<3>"),
                   kernel="k_vi_sweep_missions<3>", algorithmic_bytes_per_launch=solve_bytes / max(1, n_v // args.steps),
                   bytes_full_sweep=sweep_bytes, bytes_per_step=solve_bytes, launch_ms=sweep_s * 1e3)
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
        "vi_sweeps_per_s": sweeps_per_step * args.steps / (ms_v / 1e3),  # mission sweeps
        "vi_launches_per_s": 1e3 / (ms_v / n_v),  # fused sweeps (all missions)
        "vi_sweeps_per_step": sweeps_per_step,
        "vi_ms_per_step": ms_v / args.steps,
        "policy_ms_per_step": kt[mdp.MDP_KERNEL_POLICY][1] / args.steps,
        "copy_ms_per_step": kt[mdp.MDP_KERNEL_COPY][1] / args.steps,
        "build_shape": (None if tune is None else dict(tune["shapes"][tune["best"]], sample_layers=tune["sample_layers"],
                                                        default_ms=tune["shapes"][tune["default"]]["ms"])),
        "roofline": dominant,
        "rooflines": {"build": roof_build, "vi_sweep": roof_vi},
    }
    del model, scratch, vs, pis
    torch.cuda.empty_cache()
    if not args.no_batched:
        try:
            out["batched"] = batched_leg(pl)
        except Exception as e:  # reported, never hides the main line
            out["batched"] = {"error": repr(e)}
    if not args.no_served:
        try:
            out["served"] = served_leg(pl, args.serve_seconds, args.serve_rate, build_share=args.build_share,
                                       sweeps_per_step=args.serve_sweeps)
            out["p50_ms_served"] = out["served"]["served"]["p50_ms"]
            out["p99_ms_served"] = out["served"]["served"]["p99_ms"]
        except Exception as e:
            out["served"] = {"error": repr(e)}
    if not args.no_cpu_baseline:
        cb = cpu_baseline(w)
        out["cpu_baseline"] = cb
        out["speedup_vs_oracle_1core"] = out["build_samples_per_s"] / cb["value"]
    pl.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
