"""Benchmark of the end-to-end planning step on one MI355X.

One step = mdp_build of one instance (every (layer, cell, action) row from all
flow realizations, all requested missions from one histogram pass) + value
iteration to convergence (the instance's missions in one
mdp_value_iterate_missions solve) + mdp_policy per mission. Inputs are resident
in HBM before the timed region.

The headline step is the large instance: 200 x 200 cells, 200 layers, 16 modes,
10000 AR(1) realizations, 32 headings, 7 x 7 sub-grid, net-energy mission (the
paper's 200 x 200 x 200 shape). The paper-shaped instance (100 x 100 x 120,
5000 realizations, 16 headings, three missions) is timed the same way and
reported under "paper_shaped"; the 64-instance batch and the served trace are
reported beside.

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
FP32_VECTOR = 157.3e12                 # FP32 vector peak (FLOP/s)
# VALU lane-op rate: the fp32 vector peak counts 2 flops per FMA lane-op, so
# 157.3 TFLOP/s is 7.86e13 lane-ops/s (32 lanes per SIMD per clock); the build
# kernel has been measured above the 16-lane figure (3.93e13), which rules that
# one out as the ceiling.
VALU_LANE_OPS = FP32_VECTOR / 2         # 7.86e13 lane-ops/s
HBM_BW = 8.0e12                        # bytes/s

# Counters per launch from rocprofv3 on this benchmark (profiles/*.md), each for
# the kernel source whose sha256 prefix is given; after any change to that
# source the figure is reported null. FETCH_SIZE / WRITE_SIZE are already
# scaled to bytes by the plain-copy calibration (FETCH x2.000, WRITE x1.000);
# valu_insts is SQ_INSTS_VALU (wave instructions) per launch.
MEASURED = {
    ("k_build", "large"): dict(src="paper_2109_00857_amd/csrc/build.hip", sha256="8467cb26c0ccf1b2",
                               read=406806330, write=477817336, valu_insts=11386517926),
    ("k_build", "paper_shaped"): dict(src="paper_2109_00857_amd/csrc/build.hip", sha256="8467cb26c0ccf1b2",
                                      read=380743296, write=888004032, valu_insts=11858140138),
    ("k_vi_sweep_rows<1>", "large"): dict(src="paper_2109_00857_amd/csrc/vi.hip", sha256="b9fad8aee23f57f8",
                                          read=3165340749, write=32609961, valu_insts=279657759),
    ("k_vi_sweep_rows<3>", "paper_shaped"): dict(src="paper_2109_00857_amd/csrc/vi.hip", sha256="b9fad8aee23f57f8",
                                                 read=294722012, write=14990360, valu_insts=50547188),
}


def _src_sha(src: str) -> str:
    import hashlib

    with open(os.path.join(ROOT, src), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured(kernel: str, workload: str, field: str):
    """A counter figure per launch of this kernel on this workload, measured on the
    current kernel source, or None."""
    m = MEASURED.get((kernel, workload))
    if m is None or m.get(field) is None or _src_sha(m["src"]) != m["sha256"]:
        return None
    return m[field]


def measured_traffic(kernel: str, workload: str):
    r, w = measured(kernel, workload, "read"), measured(kernel, workload, "write")
    return None if r is None or w is None else r + w


def host_cpu() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return dict(model=model, logical_cpus=os.cpu_count(), usable_cpus=usable)


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
    cpu = host_cpu()
    return dict(value=n_samples / dt, unit="samples/s", cores=1, kind="oracle",
                sample=f"{n_rows} random (t, cell, action) rows of the {w.name} workload, "
                       f"{n_samples} realization landings, full-domain binning and fp64 rewards, "
                       f"{dt:.1f} s on one host core",
                host_cpu=cpu["model"], host_logical_cpus=cpu["logical_cpus"], host_usable_cpus=cpu["usable_cpus"])


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


def window_fits(p: dict, na: int) -> bool:
    """Whether the sweep stages a window of v(t+1) for this problem (and so reads the
    packed entries): the grid rows a block of min(512 / N_a, N_c) cells reaches,
    (S - 1) / nx + 2 + 2 h_y of them (at most ny), in 16 KB of fp64."""
    S = min(512 // na, p["nx"] * p["ny"])
    rows = min((S - 1) // p["nx"] + 2 + 2 * p["sub_hy"], p["ny"])
    return rows * p["nx"] * 8 <= 8 * 256 * 8


def packs(p: dict, na: int) -> bool:
    """Whether the build packs the model for the fused sweep: the window fits and the
    entries of a sweep block (min(512 / N_a, N_c) cells, their N_a rows of at most
    max_row entries: the sub-grid's cells, one more with the swept-path test, at most
    n_real) have 16-bit offsets."""
    nsg = (2 * p["sub_hx"] + 1) * (2 * p["sub_hy"] + 1) + (1 if p.get("flags", 0) & 2 else 0)
    S = min(512 // na, p["nx"] * p["ny"])
    return window_fits(p, na) and S * na * min(nsg, p["n_real"]) <= 0xFFFF


def skipped_fraction(w) -> float:
    """Share of the nominal samples whose source cell is the target or an obstacle
    (their rows are fixed single entries; no landing is computed for them)."""
    import numpy as np

    p = w.problem
    nc = p["nx"] * p["ny"]
    skip = np.zeros((p["nt"], nc), bool)
    skip[:, p["target_j"] * p["nx"] + p["target_i"]] = True
    if w.mask is not None:
        skip |= w.mask[:-1].reshape(p["nt"], nc).astype(bool)
    return float(skip.mean())


def rollout_leg(pl, w, p, env, pis, missions, reps: int = 3) -> dict:
    """Each mission's policy rolled out in every realization (mdp_rollout, the
    paper's Sec. IV use of the policies): ensemble statistics and the time of
    one rollout (HIP events, inputs resident)."""
    import torch

    from paper_2109_00857_amd import mdp

    nr, nt = p["n_real"], p["nt"]
    scratch = torch.empty(mdp.mdp_rollout_query(p), dtype=torch.uint8, device=pl.device)
    traj = torch.empty((nt + 1, nr), dtype=torch.int32, device=pl.device)
    st = mdp.stats_buffer(mdp.MdpRolloutStats)
    s = torch.cuda.current_stream()
    out = {}
    for m, pi in zip(missions, pis):
        ms = _ev_ms(s, lambda: mdp.mdp_rollout(pl.ctx, p, env, pi, traj, None, scratch, st, s), reps)
        torch.cuda.synchronize()
        d = mdp.rollout_stats_dict(st)
        d["ms"] = ms
        out[W_MISSIONS[m]] = d
    return out


W_MISSIONS = {0: "time", 1: "energy", 2: "net_energy"}


def replan_leg(pl, w, p, env, vs, missions, reps: int = 3) -> dict:
    """Re-planning after a forecast update at the middle layer: new coefficient
    draws for layers t >= nt/2, then mdp_build_from (those layers only) +
    mdp_value_iterate_layers (those layers only, warm-started from the solution
    before the update) + mdp_policy, against the full step on the updated
    environment (build, cold solve, policy)."""
    import numpy as np
    import torch

    from paper_2109_00857_amd import mdp

    t0 = p["nt"] // 2
    mu2 = w.mu.copy()
    rng = np.random.default_rng(2718)
    K, nr = mu2.shape[1], mu2.shape[2]
    sig = (0.2 / np.arange(1, K + 1))[:, None]
    mu2[t0:] = (sig * rng.standard_normal((p["nt"] - t0, K, nr))).astype(np.float32)
    env2 = dict(env, mu=torch.from_numpy(mu2).to(pl.device))
    m = missions[0]
    model, st2 = pl.build(p, env2)  # a model sized for the updated environment (untimed)
    assert st2["status"] == mdp.MDP_OK, st2
    scratch = pl.scratch(p)
    bst, vst = mdp.stats_buffer(mdp.MdpBuildStats), mdp.stats_buffer(mdp.MdpViStats)
    pi = torch.empty(vs[0].numel(), dtype=torch.int32, device=pl.device)
    s = torch.cuda.current_stream()
    v_prev = vs[0].clone()  # the solution before the update: the re-plan's warm start
    v = torch.empty_like(v_prev)

    def replan():
        v.copy_(v_prev)
        mdp.mdp_build_from(pl.ctx, p, env2, model, t0, scratch, bst, s)
        mdp.mdp_value_iterate_layers(pl.ctx, p, model, m, t0, 1e-6, 100000, v, scratch, vst, s)
        mdp.mdp_policy(pl.ctx, p, model, m, v, pi, s)

    def full():
        mdp.mdp_build(pl.ctx, p, env2, model, scratch, bst, s)
        v.zero_()
        mdp.mdp_value_iterate(pl.ctx, p, model, m, 1e-6, 100000, v, scratch, vst, s)
        mdp.mdp_policy(pl.ctx, p, model, m, v, pi, s)

    full()  # warm, and the model now holds the updated build
    ms_full = _ev_ms(s, full, reps)
    ms_replan = _ev_ms(s, replan, reps)
    b, vi = mdp.read_stats(bst, mdp.MdpBuildStats), mdp.read_stats(vst, mdp.MdpViStats)
    assert b["status"] == mdp.MDP_OK and vi["status"] == mdp.MDP_OK, (b, vi)
    return dict(t0=t0, mission=W_MISSIONS[m], ms_replan=ms_replan, ms_full=ms_full, speedup=ms_full / ms_replan,
                rebuilt_samples=b["samples"], sweeps=vi["sweeps"])


def step_leg(pl, w, label: str, steps: int, warmup: int, autotune: bool = True, near_edge: bool = False,
             extras: bool = False, shape=None) -> dict:
    """Time `steps` planning steps of workload w (after `warmup` untimed ones):
    build + value iteration of every mission + policies. Returns the step time,
    the per-kernel rates and the rooflines of the build and the sweep; with
    `extras`, also the policies' rollouts and a re-planning timing (untimed in
    the step)."""
    import torch

    from paper_2109_00857_amd import mdp

    p = dict(w.problem)
    if near_edge:
        p["flags"] |= mdp.MDP_FLAG_NEAR_EDGE
    missions = w.missions()
    env = pl.upload_env(w)
    tune = None
    if shape is not None:  # a given build launch shape (row lanes, realizations per chunk, 16-bit counters)
        mdp.mdp_ctx_set_plan(pl.ctx, p, *shape)
    elif autotune:
        tune = mdp.mdp_autotune(pl.ctx, p, env)  # untimed: the build launch shape
    sizes = mdp.mdp_build_query(p)
    model, st0 = pl.build(p, env)  # sizes the model (untimed)
    assert st0["status"] == mdp.MDP_OK, st0
    nnz = st0["nnz"]
    del model
    torch.cuda.empty_cache()
    model = pl.alloc_model(p, nnz, packed=True)  # with the fused sweep's packed entries
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

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    print(f"[bench] {label}: timing {steps} steps", file=sys.stderr, flush=True)
    mdp.mdp_ctx_profile(pl.ctx, True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    mdp.mdp_ctx_profile(pl.ctx, False)
    ms_step = ev0.elapsed_time(ev1) / steps
    bs = mdp.read_stats(bstat, mdp.MdpBuildStats)
    vst = [mdp.read_stats(vstat[k * vsz:(k + 1) * vsz], mdp.MdpViStats) for k in range(len(missions))]
    assert bs["status"] == mdp.MDP_OK and all(v["status"] == mdp.MDP_OK for v in vst), (bs, vst)

    kt = {k: mdp.mdp_ctx_profile_read(pl.ctx, k) for k in
          (mdp.MDP_KERNEL_BUILD, mdp.MDP_KERNEL_VI_SWEEP, mdp.MDP_KERNEL_POLICY, mdp.MDP_KERNEL_COPY)}
    n_b, ms_b = kt[mdp.MDP_KERNEL_BUILD]
    n_v, ms_v = kt[mdp.MDP_KERNEL_VI_SWEEP]
    nominal = w.nominal_samples
    K, na = p["n_modes"], w.n_actions
    rows = sizes["n_rows"]
    build_s = ms_b / 1e3 / steps            # all passes of one build
    build_launch_s = ms_b / 1e3 / n_b       # one launch (pass)
    samples_launch = nominal / bs["n_slabs"]

    # Build kernel (VALU-bound): algorithmic FP32 flops per sample are the X, Y
    # adds of the landing (2) plus the 2K + 2 FMAs (2 flops each) of velocity
    # synthesis and position per (layer, cell, realization), shared by the N_a
    # actions. The measured VALU issue rate (SQ_INSTS_VALU x 64 lanes per launch,
    # over the live launch time) is reported beside it against 7.86e13 lane-op/s.
    flops_per_sample = 2.0 + 2.0 * (2.0 * K + 2.0) / na
    ach_flops = flops_per_sample * samples_launch / build_launch_s
    kname = "k_build"
    valu = measured(kname, label, "valu_insts")
    roof_build = dict(bound="alu", achieved=ach_flops / 1e12, peak=FP32_VECTOR / 1e12, unit="TFLOP/s",
                      frac=ach_flops / FP32_VECTOR, traffic=measured_traffic(kname, label), kernel=kname,
                      fp32_flops_per_sample=flops_per_sample, samples_per_launch=samples_launch,
                      launch_ms=build_launch_s * 1e3,
                      valu_lane_ops_per_sample_issued=None if valu is None else valu * 64 / samples_launch,
                      valu_issue_frac=None if valu is None else valu * 64 / build_launch_s / VALU_LANE_OPS,
                      valu_issue_peak_Tops=VALU_LANE_OPS / 1e12)
    # VI (HBM-bound): compulsory bytes of the stored format for the layers each
    # fused sweep recomputes (sweep k of a solve recomputes layers t < nt - k + 1):
    # per layer 2 B row offset per row and 4 B per nonzero (the packed model;
    # 8 B row pointer and 6 B as col + cnt when it is not packed), read once for all
    # missions, plus per mission still iterating 4 B reward per row and v read
    # and written once per state.
    nt, nc = p["nt"], p["nx"] * p["ny"]
    rp_layer = model["row_ptr"][:: nc * na].cpu().numpy()  # row_ptr at layer starts (+ end)
    nnz_layer = rp_layer[1:] - rp_layer[:-1]
    packed = packs(p, na)
    shared_bytes = (2 if packed else 8) * nc * na + (4 if packed else 6) * nnz_layer
    mission_bytes = 4 * nc * na + 16 * nc
    solve_bytes = 0
    for k in range(max(v["sweeps"] for v in vst)):
        live = sum(1 for v in vst if v["sweeps"] > k)
        t_hi = max(0, min(nt, nt - k + 1))
        solve_bytes += int(shared_bytes[:t_hi].sum() + live * mission_bytes * t_hi)
    sweep_bytes = int(shared_bytes.sum() + len(missions) * mission_bytes * nt) + 8  # one full fused sweep
    sweep_s = ms_v / 1e3 / n_v
    ach_hbm = solve_bytes * steps / (ms_v / 1e3)
    sweeps_per_step = sum(v["sweeps"] for v in vst)
    vname = f"k_vi_sweep_rows<{len(missions)}>" if packed else f"k_vi_sweep_missions<{len(missions)}>"
    roof_vi = dict(bound="hbm", achieved=ach_hbm / 1e9, peak=HBM_BW / 1e9, unit="GB/s", frac=ach_hbm / HBM_BW,
                   traffic=measured_traffic(vname, label), kernel=vname,
                   bytes_per_nonzero=4 if packed else 6,
                   algorithmic_bytes_per_launch=solve_bytes / max(1, n_v // steps), bytes_full_sweep=sweep_bytes,
                   bytes_per_step=solve_bytes, launch_ms=sweep_s * 1e3)
    out = dict(
        workload=w.name, rows=rows, nnz=nnz, samples_per_step=nominal, missions=missions,
        skipped_source_fraction=skipped_fraction(w), near_edge_counted=bool(near_edge),
        ms_per_step=ms_step, samples_per_s=nominal / (ms_step / 1e3),
        build_samples_per_s=nominal / build_s, build_ms=build_s * 1e3, build_launches_per_step=n_b // steps,
        vi_sweeps_per_s=sweeps_per_step * steps / (ms_v / 1e3),  # mission sweeps
        vi_launches_per_s=1e3 / (ms_v / n_v),  # fused sweeps (all missions)
        vi_sweeps_per_step=sweeps_per_step, vi_ms_per_step=ms_v / steps,
        policy_ms_per_step=kt[mdp.MDP_KERNEL_POLICY][1] / steps, copy_ms_per_step=kt[mdp.MDP_KERNEL_COPY][1] / steps,
        build_shape=(dict(zip(("row_lanes", "rch", "pack16"), shape), given=True) if shape is not None else
                     None if tune is None else dict(tune["shapes"][tune["best"]], sample_layers=tune["sample_layers"],
                                                    default_ms=tune["shapes"][tune["default"]]["ms"])),
        rooflines={"build": roof_build, "vi_sweep": roof_vi},
        dominant="build" if ms_b >= ms_v else "vi_sweep",
    )
    if extras:
        out["rollouts"] = rollout_leg(pl, w, p, env, pis, missions)
        if len(missions) == 1:
            out["replan"] = replan_leg(pl, w, p, env, vs, missions)
        if not near_edge:  # the build with near-edge counting on (untimed in the step)
            pn = dict(p, flags=p["flags"] | mdp.MDP_FLAG_NEAR_EDGE)
            ms_near = _ev_ms(stream, lambda: mdp.mdp_build(pl.ctx, pn, env, model, scratch, bstat, stream), 2)
            bn = mdp.read_stats(bstat, mdp.MdpBuildStats)
            assert bn["status"] == mdp.MDP_OK, bn
            out["build_near_edge"] = dict(ms=ms_near, ms_without=build_s * 1e3, n_near_edge=bn["n_near_edge"],
                                          near_edge_fraction=bn["n_near_edge"] / max(bn["samples"], 1))
    del model, scratch, vi_scratch, vs, pis
    torch.cuda.empty_cache()
    return out


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

    large = np.array([w.name.startswith("c2") for w, _ in reqs])

    def stats(lat, wall):
        a = np.array([lat[j] for j in range(n)]) * 1e3
        by_class = {}
        for cls, sel in (("paper_shaped", large), ("batched_mix", ~large)):
            if sel.any():
                by_class[cls] = dict(n=int(sel.sum()), p50_ms=float(np.percentile(a[sel], 50)),
                                     p99_ms=float(np.percentile(a[sel], 99)), mean_ms=float(a[sel].mean()))
        return dict(p50_ms=float(np.percentile(a, 50)), p99_ms=float(np.percentile(a, 99)),
                    mean_ms=float(a.mean()), max_ms=float(a.max()), wall_s=wall,
                    requests_per_s=n / wall, samples_per_s=samples / wall, by_class=by_class)

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
    print(f"[bench] served: {n} requests over {seconds:.0f} s", file=sys.stderr, flush=True)
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
    print("[bench] served trace: sequential plain solves", file=sys.stderr, flush=True)
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


HEADLINE = "large"


def workload(name: str):
    from paper_2109_00857_amd import workloads as W

    if name == "paper_actions":  # the paper's application action set: 16 headings x 2 speeds
        w = W.config2()
        w.problem["n_speed"] = 2
        w.name = "c2_paper_actions"
        return w
    return {"large": W.config3, "paper_shaped": W.config2}[name]()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["large", "paper_shaped"], default=HEADLINE,
                    help="instance of the headline step (default: the 200x200x200 large instance)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--near-edge", action="store_true", help="also count near-edge samples")
    ap.add_argument("--no-second", action="store_true", help="skip the second single-instance workload")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-instance batched leg")
    ap.add_argument("--no-served", action="store_true", help="skip the served-trace leg")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="length of the served trace")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="request arrival rate (per second)")
    ap.add_argument("--serve-rate-high", type=float, default=60.0,
                    help="arrival rate of a second, shorter served trace at a higher load (0: skip)")
    ap.add_argument("--serve-seconds-high", type=float, default=20.0, help="length of the higher-load trace")
    ap.add_argument("--build-share", type=int, default=100,
                    help="percent of the GPU's resident workgroups a served build batch may hold")
    ap.add_argument("--serve-sweeps", type=int, default=32, help="most sweeps per served scheduler step")
    ap.add_argument("--no-autotune", action="store_true", help="build with the default launch shape")
    ap.add_argument("--shape", type=str, default=None,
                    help="build launch shape ROW_LANES,RCH,PACK16 for the headline workload instead of the "
                         "autotuner's pick (e.g. to profile the tuned kernel without the tuner's launches)")
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

    from paper_2109_00857_amd import mdp

    pl = mdp.Planner(0)
    w = workload(args.workload)
    print(f"[bench] headline workload {args.workload}: {w.n_rows} rows, {w.nominal_samples:.3e} samples",
          file=sys.stderr, flush=True)
    shape = None if args.shape is None else tuple(int(x) for x in args.shape.split(","))
    main_leg = step_leg(pl, w, args.workload, args.steps, args.warmup, autotune=not args.no_autotune,
                        near_edge=args.near_edge, extras=not args.no_second, shape=shape)
    rf = main_leg["rooflines"]
    descr = {"large": "large single instance: 200x200 cells, 200 layers, 16 modes, 10000 AR(1) realizations, "
                      "32 headings, 7x7 sub-grid, 4 moving discs, net-energy mission",
             "paper_shaped": "paper-shaped single instance: 100x100 cells, 120 layers, 10 modes, 5000 AR(1) "
                             "realizations, 16 headings, 5x5 sub-grid, 4 moving discs, time + energy + net-energy "
                             "missions"}
    out = {
        "metric": "MDP build samples/s + VI sweeps/s (% roofline); p50/p99 plan latency served",
        "value": main_leg["samples_per_s"],
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 landings, f64 values",
        "data": "synthetic",
        "config": {"workload": descr[args.workload], "rows": main_leg["rows"], "nnz": main_leg["nnz"],
                   "samples_per_step": main_leg["samples_per_step"],
                   "skipped_source_fraction": main_leg["skipped_source_fraction"],
                   "near_edge_counted": main_leg["near_edge_counted"]},
        "build_samples_per_s": main_leg["build_samples_per_s"],
        "build_ms": main_leg["build_ms"],
        "vi_sweeps_per_s": main_leg["vi_sweeps_per_s"],
        "vi_launches_per_s": main_leg["vi_launches_per_s"],
        "vi_sweeps_per_step": main_leg["vi_sweeps_per_step"],
        "vi_ms_per_step": main_leg["vi_ms_per_step"],
        "policy_ms_per_step": main_leg["policy_ms_per_step"],
        "copy_ms_per_step": main_leg["copy_ms_per_step"],
        "build_shape": main_leg["build_shape"],
        "roofline": rf[main_leg["dominant"]],
        "rooflines": rf,
    }
    for k in ("rollouts", "replan", "build_near_edge"):
        if k in main_leg:
            out[k] = main_leg[k]
    if not args.no_second:
        other = "paper_shaped" if args.workload == "large" else "large"
        for name in (other, "paper_actions"):
            try:
                out[name] = step_leg(pl, workload(name), name, args.steps, args.warmup,
                                     autotune=not args.no_autotune, near_edge=args.near_edge, extras=True)
            except Exception as e:  # reported, never hides the main line
                out[name] = {"error": repr(e)}
    if not args.no_batched:
        try:
            out["batched"] = batched_leg(pl)
        except Exception as e:
            out["batched"] = {"error": repr(e)}
    if not args.no_served:
        try:
            out["served"] = served_leg(pl, args.serve_seconds, args.serve_rate, build_share=args.build_share,
                                       sweeps_per_step=args.serve_sweeps)
            out["p50_ms_served"] = out["served"]["served"]["p50_ms"]
            out["p99_ms_served"] = out["served"]["served"]["p99_ms"]
        except Exception as e:
            out["served"] = {"error": repr(e)}
        if args.serve_rate_high > 0:
            try:
                out["served_high_load"] = served_leg(pl, args.serve_seconds_high, args.serve_rate_high,
                                                     build_share=args.build_share, sweeps_per_step=args.serve_sweeps)
            except Exception as e:
                out["served_high_load"] = {"error": repr(e)}
    if not args.no_cpu_baseline:
        cb = cpu_baseline(w)
        out["cpu_baseline"] = cb
        out["speedup_vs_oracle_1core"] = out["build_samples_per_s"] / cb["value"]
    pl.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
