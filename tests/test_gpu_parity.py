"""HIP path vs CPU oracle, through the C ABI (needs an MI355X)."""
import json
import os

import numpy as np
import pytest

from paper_2109_00857_amd import workloads as W

from gpu_helpers import (REL_TOL, assert_counts_equal, assert_policy_optimal, assert_rewards_close,
                         assert_values_close, model_to_host)

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def planner():
    import torch

    assert torch.cuda.is_available()
    from paper_2109_00857_amd import mdp

    pl = mdp.Planner(0)
    yield pl
    pl.close()


def _build_both(planner, ora, w, near=True):
    from paper_2109_00857_amd import mdp

    p = dict(w.problem)
    if near:
        p["flags"] |= mdp.MDP_FLAG_NEAR_EDGE
    env = planner.upload_env(w)
    model, stats = planner.build(p, env)
    om = ora.build_model(w)
    return p, env, model, stats, om


def _full_parity(planner, ora, w, label):
    import torch

    print(f"[parity] {label}: {w.problem['nx']}x{w.problem['ny']}x{w.problem['nt']} "
          f"Nr={w.problem['n_real']} Na={w.n_actions}", flush=True)
    p, env, model, stats, om = _build_both(planner, ora, w)
    assert stats["status"] == 0, stats
    assert stats["n_escape"] == om["n_escape"] == 0
    assert stats["n_near_edge"] == om["n_near_edge"]
    g = model_to_host(model, stats)
    assert stats["nnz"] == om["nnz"]
    nc = w.problem["nx"] * w.problem["ny"]
    src = np.arange(w.n_states) % nc
    skipped = (src == w.problem["target_j"] * w.problem["nx"] + w.problem["target_i"])
    if w.mask is not None:
        skipped |= w.mask[:-1].reshape(-1).astype(bool)
    assert stats["samples"] == int((~skipped).sum()) * w.n_actions * w.problem["n_real"]
    assert_counts_equal(g, om)
    missions = w.missions()
    assert_rewards_close(g, om, missions)
    for m in missions:
        v, vst = planner.value_iterate(p, model, m, tol=1e-6)
        assert vst["status"] == 0 and vst["sweeps"] <= w.problem["nt"] + 1, vst
        v = v.cpu().numpy()
        v_ora, pi_ora, w_ora = ora.backward(w, om, m)
        assert_values_close(v, v_ora, w_ora)
        pi = planner.policy(p, model, m, torch.from_numpy(v).to(planner.device))
        rate = assert_policy_optimal(ora, w, om, m, v_ora, w_ora, pi.cpu().numpy())
        print(f"[parity] {label} mission {m}: sweeps={vst['sweeps']} policy match={rate:.4f}", flush=True)
    return p, env, model, stats, om


@pytest.mark.parametrize("case", [0, 1])
def test_worked_example(planner, ora, case):
    with open(os.path.join(GOLDEN, "worked_example_uniform_flow.json")) as f:
        g = json.load(f)
    c = g["cases"][case]
    s = g["setup"]
    w = W.uniform_flow(s["nx"], s["ny"], c["nt"], s["u0"], s["v0"], n_real=8, n_head=s["n_head"],
                       f_max=s["f_max"], dx=s["dx"], dy=s["dy"], dt=s["dt"], start=tuple(s["start"]),
                       target=tuple(s["target"]), sub_h=2)
    p, env, model, stats, om = _full_parity(planner, ora, w, f"worked example T={c['nt']}")
    v, _ = planner.value_iterate(p, model, 0)
    pi = planner.policy(p, model, 0, v).cpu().numpy()
    v = v.cpu().numpy()
    nx, ny = s["nx"], s["ny"]
    for st in c["states"]:
        k = (st["t"] * ny + st["j"]) * nx + st["i"]
        assert v[k] == st["v"] and pi[k] == st["pi"], st


def test_c1_full(planner, ora):
    """Config 1 as specified, sub-grid sized on the device and checked against the oracle."""
    from paper_2109_00857_amd import mdp

    w = W.config1()
    env = planner.upload_env(w)
    hx, hy = mdp.mdp_subgrid_auto(planner.ctx, w.problem, env)
    assert (hx, hy) == ora.subgrid_auto(w)
    w.problem["sub_hx"], w.problem["sub_hy"] = hx, hy
    _full_parity(planner, ora, w, f"c1 (h={hx},{hy})")


def test_c2_shape_ragged(planner, ora):
    """Config-2 shapes (16 headings, 10 trig modes, AR(1), discs, all missions) on a
    ragged grid and realization count that span many tiles and chunks."""
    w = W.config2(nx=37, ny=29, nt=4, n_real=1000)
    _full_parity(planner, ora, w, "c2-shaped ragged")


def test_c3_shape_ragged(planner, ora):
    """Config-3 shapes (32 headings, 16 modes, 7x7 sub-grid, net energy), ragged."""
    w = W.config3(nx=23, ny=19, nt=3, n_real=700)
    _full_parity(planner, ora, w, "c3-shaped ragged")


def test_time_varying_fields_and_speeds(planner, ora):
    """Time-varying mean and modes, two speeds, few modes (other kernel variants)."""
    w = W.config2(nx=21, ny=18, nt=3, n_real=300, K=3, n_head=6)
    rng = np.random.default_rng(3)
    nt = w.problem["nt"]
    w.ubar = np.ascontiguousarray(np.repeat(w.ubar, nt, 0) * rng.uniform(0.5, 1.5, (nt, 1, 1)).astype(np.float32))
    w.vbar = np.ascontiguousarray(rng.normal(0, 0.05, w.ubar.shape).astype(np.float32))
    w.phiu = np.ascontiguousarray(np.repeat(w.phiu, nt, 0) * rng.uniform(0.8, 1.2, (nt, 1, 1, 1)).astype(np.float32))
    w.phiv = np.ascontiguousarray(np.repeat(w.phiv, nt, 0))
    w.problem.update(mean_time_varying=1, mode_time_varying=1, n_speed=2, sub_hx=3, sub_hy=3)
    w.problem["f_max"] = 0.25
    w.check()
    _full_parity(planner, ora, w, "time-varying, 2 speeds")


def test_gaussian_bins_bitexact(planner, ora):
    """The closed-form stochastic uniform-flow instance with 50000 realizations."""
    w = W.uniform_flow(7, 7, 2, 0.25, 0.0, n_real=50000, n_head=4, f_max=0.6, sigma=0.2,
                       start=(0, 0), target=(6, 6), sub_h=3, seed=11)
    _full_parity(planner, ora, w, "gaussian bins")


@pytest.mark.parametrize("h", [0, 1])
def test_escape_detection(planner, ora, h):
    """Too small a sub-grid: MDP_E_SUBGRID with the oracle's exact escape count."""
    from paper_2109_00857_amd import mdp

    w = W.config1(nt=3, n_real=200, sub_h=h)
    p, env, model, stats, om = _build_both(planner, ora, w)
    assert om["n_escape"] > 0
    assert stats["status"] == mdp.MDP_E_SUBGRID
    assert stats["n_escape"] == om["n_escape"]


def test_capacity_too_small(planner, ora):
    from paper_2109_00857_amd import mdp

    w = W.config1(nt=3, n_real=100, sub_h=3)
    env = planner.upload_env(w)
    model = planner.alloc_model(w.problem, 1000)
    scratch = planner.scratch(w.problem)
    st = mdp.stats_buffer(mdp.MdpBuildStats)
    mdp.mdp_build(planner.ctx, w.problem, env, model, scratch, st)
    import torch

    torch.cuda.synchronize()
    s = mdp.read_stats(st, mdp.MdpBuildStats)
    om = ora.build_model(w)
    assert s["status"] == mdp.MDP_E_CAPACITY and s["nnz"] == om["nnz"] > 1000
    np.testing.assert_array_equal(model["row_ptr"].cpu().numpy(), om["row_ptr"])


def test_repeatable_bitwise(planner, ora):
    w = W.config2(nx=30, ny=30, nt=3, n_real=500)
    env = planner.upload_env(w)
    m1, s1 = planner.build(w.problem, env)
    m2, s2 = planner.build(w.problem, env)
    assert s1 == s2
    for k in ("row_ptr", "col", "cnt", "reward"):
        assert (m1[k].view(-1).cpu().numpy().tobytes() == m2[k].view(-1).cpu().numpy().tobytes()), k
    v1, _ = planner.value_iterate(w.problem, m1, 0)
    v2, _ = planner.value_iterate(w.problem, m2, 0)
    assert v1.cpu().numpy().tobytes() == v2.cpu().numpy().tobytes()


def test_vi_layered_residual(planner, ora):
    """Jacobi from v0 = 0 reaches residual exactly 0 within nt + 1 sweeps; with
    tol = 0 it runs exactly max_sweeps and the values do not move."""
    w = W.config1(nt=6, n_real=100, sub_h=3)
    env = planner.upload_env(w)
    model, stats = planner.build(w.problem, env)
    v, st = planner.value_iterate(w.problem, model, 0, tol=1e-300)
    assert st["status"] == 0 and st["residual"] == 0.0 and st["sweeps"] <= 7
    v2, st2 = planner.value_iterate(w.problem, model, 0, tol=0.0, max_sweeps=9)
    assert st2["sweeps"] == 9 and st2["status"] != 0
    assert v.cpu().numpy().tobytes() == v2.cpu().numpy().tobytes()


def test_vi_partial_sweeps_and_warm_start(planner, ora):
    """k synchronous sweeps (k < nt + 1, so layers are still moving) match the
    oracle's k Jacobi sweeps, and a random warm start converges to the cold
    start's values bit for bit within nt + 1 sweeps (every layer's final value
    depends only on the model, whatever v0 was)."""
    import torch

    w = W.config1(nt=8, n_real=200, sub_h=3)
    env = planner.upload_env(w)
    model, stats = planner.build(w.problem, env)
    om = ora.build_model(w)
    _, _, w_ora = ora.backward(w, om, 0)
    for k in (1, 2, 4, 7):
        v_gpu, st = planner.value_iterate(w.problem, model, 0, tol=0.0, max_sweeps=k)
        assert st["sweeps"] == k
        v_ora, k_ora, _ = ora.jacobi(w, om, 0, tol=0.0, max_sweeps=k)
        assert k_ora == k
        err = np.abs(v_gpu.cpu().numpy() - v_ora)
        assert (err <= 1e-5 * (w_ora + 1.0)).all(), (k, float(err.max()))
    v_cold, st_cold = planner.value_iterate(w.problem, model, 0)
    rng = np.random.default_rng(5)
    v0 = torch.from_numpy(rng.normal(0.0, 100.0, w.n_states)).to(planner.device)
    v_warm, st_warm = planner.value_iterate(w.problem, model, 0, v0=v0)
    assert st_cold["status"] == 0 and st_warm["status"] == 0
    assert st_warm["sweeps"] <= w.problem["nt"] + 1
    assert v_warm.cpu().numpy().tobytes() == v_cold.cpu().numpy().tobytes()


def test_vi_missions_fused_equals_single(planner, ora):
    """One fused solve over several missions of a model gives each mission the
    values and stats of its own mdp_value_iterate, bit for bit: cold and warm
    starts, a sweep limit below convergence, and subsets of the missions."""
    import torch

    w = W.config2(nx=37, ny=29, nt=5, n_real=600)
    env = planner.upload_env(w)
    model, stats = planner.build(w.problem, env)
    assert stats["status"] == 0
    missions = w.missions()
    assert len(missions) == 3
    rng = np.random.default_rng(9)
    warm = [torch.from_numpy(rng.normal(0.0, 50.0, w.n_states)).to(planner.device) for _ in missions]
    cases = [(missions, None, 1e-6, 100000), (missions, warm, 1e-6, 100000), (missions, None, 0.0, 3),
             (missions[1:], None, 1e-6, 100000), (missions[::-1][:2], warm[:2], 1e-6, 100000),
             (missions[:1], None, 1e-6, 100000)]
    for ms, v0s, tol, mx in cases:
        print(f"[parity] fused missions {ms} warm={v0s is not None} tol={tol} max={mx}", flush=True)
        vs, sts = planner.value_iterate_missions(w.problem, model, ms, tol=tol, max_sweeps=mx, v0s=v0s)
        for i, m in enumerate(ms):
            v1, st1 = planner.value_iterate(w.problem, model, m, tol=tol, max_sweeps=mx,
                                            v0=None if v0s is None else v0s[i])
            assert sts[i] == st1, (ms, i, sts[i], st1)
            assert vs[i].cpu().numpy().tobytes() == v1.cpu().numpy().tobytes(), (ms, i)
    # and the fused values are the oracle's
    om = ora.build_model(w)
    vs, _ = planner.value_iterate_missions(w.problem, model, missions)
    for i, m in enumerate(missions):
        v_ora, _, w_ora = ora.backward(w, om, m)
        assert_values_close(vs[i].cpu().numpy(), v_ora, w_ora)


@pytest.mark.parametrize("shape", ["whole_rows", "narrow"])
def test_packed_entries(planner, ora, shape):
    """The build's packed entries for the fused sweep: each nonzero's
    (window index << 16) | count, the index taken in the grid rows of layer t+1
    that the sweep stages for the block of cells holding the row (0xFFFF for
    DEAD and TARGET, and every state column lies inside its window; a block
    inside one grid row stages only the columns it can reach, others whole
    rows), and each row's first entry relative to its block's first entry in
    16 bits; the fused solve reads them and gives the same values as from
    row_ptr / col / cnt, bit for bit. Blocks of 32 cells straddle some of the
    37-cell rows."""
    import torch

    if shape == "whole_rows":  # 32-cell blocks against 37-cell rows: whole-row windows
        w = W.config2(nx=37, ny=29, nt=5, n_real=600)
    else:  # 16-cell blocks (32 headings) in 150-cell rows: narrow windows
        w = W.config2(nx=150, ny=12, nt=4, n_real=300, K=4, n_head=32)
    p = w.problem
    model, st = planner.build(p, planner.upload_env(w))
    assert st["status"] == 0 and "ent" in model and "roff" in model
    nnz = st["nnz"]
    rp = model["row_ptr"].cpu().numpy()
    col = model["col"][:nnz].cpu().numpy().astype(np.int64)
    cnt = model["cnt"][:nnz].cpu().numpy().astype(np.int64)
    ent = model["ent"][:nnz].cpu().numpy().view(np.uint32).astype(np.int64)
    nx, ny, nt, hx, hy = p["nx"], p["ny"], p["nt"], p["sub_hx"], p["sub_hy"]
    nc, na, ns = nx * ny, w.n_actions, w.n_states
    S = min(512 // na, nc)
    row = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    t, c = divmod(row // na, nc)
    c0 = c // S * S
    nst = np.minimum(S, nc - c0)
    j0, j1 = c0 // nx, (c0 + nst - 1) // nx
    jw0 = np.maximum(0, j0 - hy)
    rows = np.minimum(ny - 1, j1 + hy) - jw0 + 1
    # a block inside one grid row stages only the columns it can reach, when
    # those are at most a quarter of a row
    one_row = (j0 == j1) & (4 * (S + 2 * hx) <= nx)
    iw0 = np.where(one_row, np.maximum(0, c0 - j0 * nx - hx), 0)
    cols = np.where(one_row, np.minimum(nx - 1, c0 + nst - 1 - j0 * nx + hx) - iw0 + 1, nx)
    jj, ii = divmod(col - (t + 1) * nc, nx)
    r, k = jj - jw0, ii - iw0
    inside = (t + 1 < nt) & (col < ns) & (r >= 0) & (r < rows) & (k >= 0) & (k < cols)
    assert np.all(inside | (col >= ns)), "a state column outside its window"
    assert one_row.any() == (4 * (S + 2 * hx) <= nx) and not one_row.all()
    code = np.where(inside, r * cols + k, 0xFFFF)
    np.testing.assert_array_equal(ent, code << 16 | cnt)
    rt, rc = divmod(np.arange(len(rp) - 1) // na, nc)
    first = (rt * nc + rc // S * S) * na
    np.testing.assert_array_equal(model["roff"].cpu().numpy().view(np.uint16).astype(np.int64), rp[:-1] - rp[first])
    unpacked = {k: v for k, v in model.items() if k not in ("ent", "roff")}
    vs, sts = planner.value_iterate_missions(p, model, w.missions())
    vu, stu = planner.value_iterate_missions(p, unpacked, w.missions())
    assert sts == stu
    for a, b in zip(vs, vu):
        assert torch.equal(a, b)


def test_blocks_too_large_to_pack(planner):
    """A 13x13 sub-grid (rows of up to 169 entries) with 400 realizations and 8
    headings: a sweep block (64 cells x 8 actions) may hold more entries than
    16-bit offsets reach, so the build leaves the packed buffers untouched and
    the fused solve reads row_ptr / col / cnt; same values as the unpacked
    model. ent without roff is refused."""
    import torch

    from paper_2109_00857_amd import mdp

    w = W.config1(nt=4, n_real=400, sub_h=6)
    p = w.problem
    env = planner.upload_env(w)
    ref, st = planner.build(p, env, packed=False)
    assert st["status"] == 0
    model = planner.alloc_model(p, st["nnz"], packed=True)
    model["ent"].fill_(-1)
    model["roff"].view(torch.int16).fill_(7)
    sbuf = mdp.stats_buffer(mdp.MdpBuildStats)
    scratch = planner.scratch(p)
    mdp.mdp_build(planner.ctx, p, env, model, scratch, sbuf)
    assert mdp.mdp_build_sync(planner.ctx, sbuf) == mdp.MDP_OK
    assert bool((model["ent"] == -1).all()) and bool((model["roff"].view(torch.int16) == 7).all())
    for k in ("row_ptr", "col", "cnt", "reward"):
        assert torch.equal(model[k], ref[k]), k
    vs, sts = planner.value_iterate_missions(p, model, w.missions())
    vr, str_ = planner.value_iterate_missions(p, ref, w.missions())
    assert sts == str_ and all(torch.equal(a, b) for a, b in zip(vs, vr))
    half = {k: v for k, v in model.items() if k != "roff"}
    with pytest.raises(mdp.MdpError) as e:
        mdp.mdp_build(planner.ctx, p, env, half, scratch, sbuf)
    assert e.value.status == mdp.MDP_E_INVALID
    with pytest.raises(mdp.MdpError) as e:
        planner.value_iterate_missions(p, half, w.missions())
    assert e.value.status == mdp.MDP_E_INVALID


def test_vi_missions_rejects_bad_arguments(planner):
    """Argument errors of the fused solve come back synchronously as MDP_E_INVALID
    (or MDP_E_SCRATCH) and enqueue nothing."""
    import torch

    from paper_2109_00857_amd import mdp

    w = W.config1(nt=3, n_real=100, sub_h=3)
    w.problem["mission_mask"] = 0b011  # missions 0 and 1 built
    model, stats = planner.build(w.problem, planner.upload_env(w))
    assert stats["status"] == 0
    ns = w.n_states
    sc = torch.empty(3 * mdp.mdp_build_query(w.problem)["scratch_bytes"], dtype=torch.uint8,
                     device=planner.device)
    st = torch.zeros(3 * mdp.C.sizeof(mdp.MdpViStats), dtype=torch.uint8, pin_memory=True)
    vs = [torch.zeros(ns, dtype=torch.float64, device=planner.device) for _ in range(4)]
    cases = [([], mdp.MDP_E_INVALID),                  # no mission
             ([0, 1, 0, 1], mdp.MDP_E_INVALID),        # more than three
             ([0, 0], mdp.MDP_E_INVALID),              # repeated mission
             ([0, 2], mdp.MDP_E_INVALID)]              # mission 2 was not built
    for ms, want in cases:
        with pytest.raises(mdp.MdpError) as e:
            mdp.mdp_value_iterate_missions(planner.ctx, w.problem, model, ms, 1e-6, 100, vs[:len(ms)], sc, st)
        assert e.value.status == want, (ms, e.value)
    with pytest.raises(mdp.MdpError) as e:  # one value buffer for two missions
        mdp.mdp_value_iterate_missions(planner.ctx, w.problem, model, [0, 1], 1e-6, 100, [vs[0], vs[0]], sc, st)
    assert e.value.status == mdp.MDP_E_INVALID
    with pytest.raises(mdp.MdpError) as e:  # scratch for one mission only
        mdp.mdp_value_iterate_missions(planner.ctx, w.problem, model, [0, 1], 1e-6, 100, vs[:2], sc[:1024], st)
    assert e.value.status == mdp.MDP_E_SCRATCH
    vs2, sts = planner.value_iterate_missions(w.problem, model, [1, 0])
    assert all(s["status"] == 0 for s in sts)


def test_wide_grid_without_window(planner, ora):
    """A grid too wide for the staged window of v(t + 1) (six grid rows of 520
    cells exceed its 16 KB): the sweeps and the policy gather every successor's
    value from memory; full parity, and the fused solve equals the single one."""
    import torch

    w = W.config2(nx=520, ny=7, nt=4, n_real=300, K=4, n_head=8)
    p, env, model, stats, om = _full_parity(planner, ora, w, "wide grid, no window")
    vs, _ = planner.value_iterate_missions(p, model, w.missions())
    for m, v in zip(w.missions(), vs):
        v1, _ = planner.value_iterate(p, model, m)
        assert torch.equal(v, v1), m


@pytest.mark.parametrize("n_head", [5, 2])
def test_unpaired_action_sets(planner, ora, n_head):
    """Action sets the paired landing loop does not take (an odd N_a; two
    headings whose x displacements differ): the build keeps one row per lane
    with 16-bit counters; full parity with the oracle."""
    from gpu_helpers import landing_loop

    w = W.config2(nx=19, ny=17, nt=4, n_real=400, K=4, n_head=n_head, missions=(0, 1))
    assert landing_loop(w.problem) == "rows"
    _full_parity(planner, ora, w, f"{n_head} headings")


def test_paper_action_set_two_speeds(planner, ora):
    """The paper's application action set, 16 headings x 2 speeds, on config-2
    shapes with all three missions (ragged grid): full parity."""
    w = W.config2(nx=33, ny=27, nt=5, n_real=800, n_head=16)
    w.problem["n_speed"] = 2
    assert w.n_actions == 32
    _full_parity(planner, ora, w, "16 headings x 2 speeds")


@pytest.mark.parametrize("n_head,n_speed,shapes,loop", [
    (32, 1, [(256, 256), (128, 256), (64, 128)], "pairs"),
    (16, 2, [(128, 256), (256, 64)], "pairs"),
    (8, 1, [(256, 64), (128, 128), (64, 256)], "pairs"),
    (4, 1, [(256, 64), (64, 128)], "pairs"),
    (5, 1, [(256, 64), (64, 128)], "rows"),
])
def test_landing_loops_at_every_row_lane_count(planner, ora, n_head, n_speed, shapes, loop):
    """The paired landing loop (two rows of a pair of actions per lane, 256 / hw
    realization parts; waves of pairs sharing Hx and waves holding the other
    pairs) and the row-per-lane loop at launch shapes with 256, 128 and 64 row
    lanes (2, 4 and 8 parts): every shape's model is the oracle's (counts
    bit-exact, rewards within the tolerance)."""
    from paper_2109_00857_amd import mdp

    from gpu_helpers import landing_loop

    w = W.config2(nx=29, ny=23, nt=3, n_real=700, K=4, n_head=n_head, missions=(0, 2))
    w.problem["n_speed"] = n_speed
    p = w.problem
    assert landing_loop(p) == loop
    om = ora.build_model(w)
    env = planner.upload_env(w)
    try:
        for rl, rch in shapes:
            print(f"[loops] {n_head}x{n_speed} ({loop}) shape ({rl}, {rch})", flush=True)
            mdp.mdp_ctx_set_plan(planner.ctx, p, rl, rch, 1)
            model, st = planner.build(p, env)
            assert st["status"] == 0 and st["nnz"] == om["nnz"], st
            g = model_to_host(model, st)
            assert_counts_equal(g, om)
            assert_rewards_close(g, om, w.missions())
    finally:
        mdp.mdp_ctx_set_plan(planner.ctx, p, 0, 0, 0)


@pytest.mark.parametrize("case", [0, 1, 2])
def test_two_speed_corridor(planner, ora, case):
    """The hand-derived two-speed corridor (slow when the horizon allows, fast
    when it must) on the GPU: its values and start actions."""
    with open(os.path.join(GOLDEN, "two_speed_corridor.json")) as f:
        g = json.load(f)
    s, c = g["setup"], g["cases"][case]
    w = W.uniform_flow(s["nx"], s["ny"], c["nt"], s["u0"], s["v0"], n_real=8, n_head=s["n_head"], f_max=s["f_max"],
                       dx=s["dx"], dy=s["dy"], dt=s["dt"], start=tuple(s["start"]), target=tuple(s["target"]),
                       sub_h=2, n_speed=s["n_speed"], mission_mask=3)
    p, env, model, stats, om = _full_parity(planner, ora, w, f"two-speed corridor case {case}")
    v, _ = planner.value_iterate(p, model, c["mission"])
    pi = planner.policy(p, model, c["mission"], v).cpu().numpy()
    s0 = s["start"][1] * s["nx"] + s["start"][0]
    # rewards are stored in fp32 (99.36 = r_term - 0.64 is not a float), so the
    # start value holds within the value tolerance of the rewards' scale
    _, _, w_ora = ora.backward(w, om, c["mission"])
    assert abs(float(v[s0]) - c["v_start"]) <= REL_TOL * w_ora[s0], (float(v[s0]), c["v_start"], w_ora[s0])
    assert pi[s0] == c["pi_start"]


def test_swept_path_obstacles(planner, ora):
    """The swept-path obstacle test (MDP_FLAG_SWEPT_PATH) with moving discs, two
    speeds and long steps, against the oracle: full parity, and some samples do
    move to DEAD compared with the landing-cell test alone."""
    from paper_2109_00857_amd import mdp

    w = W.config2(nx=30, ny=26, nt=4, n_real=500, K=4, n_head=8)
    w.problem.update(n_speed=2, f_max=0.9, sub_hx=4, sub_hy=4)
    om_plain = ora.build_model(w)
    w.problem["flags"] |= mdp.MDP_FLAG_SWEPT_PATH
    p, env, model, stats, om = _full_parity(planner, ora, w, "swept path")
    ns = w.n_states
    dead_plain = int(om_plain["cnt"][om_plain["col"] == ns].sum())
    dead_swept = int(om["cnt"][om["col"] == ns].sum())
    assert dead_swept > dead_plain, (dead_swept, dead_plain)
    with pytest.raises(mdp.MdpError):
        mdp.Batch(planner, [p], [env], [0])
