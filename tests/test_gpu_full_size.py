"""Full-size parity on sampled outputs (needs an MI355X): the paper-shaped
(100x100x120, 5000 realizations, 16 headings, three missions) and large
(200x200x200, 10000 realizations, 32 headings, 7x7 sub-grid) instances are
built and solved in the launch configuration the benchmark times (autotuned
build shape), then checked against the oracle computed one row at a time:

- sampled rows: counts bit-exact, rewards within 1e-5 of the row's expected
  |reward| (the oracle's), no sub-grid escapes;
- sampled states: one Bellman step with the oracle's rows and the GPU's values
  of the next layer reproduces the GPU's value, and the GPU's action attains
  the oracle's maximum, both within 1e-5 of the state's absolute scale
  max_a E|r| + sum P |v(s')| (the whole oracle backward pass is out of reach
  at these sizes, so the value test is the Bellman identity at any size);
- for the paper-shaped instance also the oracle's exact solution at 100
  sampled states (tests/golden/paper_shaped_values.json, written by
  tests/golden/make_paper_shaped_values.py from the oracle alone): values
  within 1e-5 of the absolute-reward value, the GPU policy's action within the
  same bound of the oracle's maximum Q."""
import json
import os

import numpy as np
import pytest

from paper_2109_00857_amd import workloads as W

from gpu_helpers import REL_TOL

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

pytestmark = pytest.mark.gpu

N_ROWS = 300
N_STATES = 120


@pytest.fixture(scope="module")
def planner():
    import torch

    assert torch.cuda.is_available()
    from paper_2109_00857_amd import mdp

    pl = mdp.Planner(0)
    yield pl
    pl.close()


def _rows_of(model, rows):
    rp = model["row_ptr"]
    import torch

    idx = torch.as_tensor(np.concatenate([rows, rows + 1]), device=rp.device)
    b = rp[idx].cpu().numpy()
    lo, hi = b[: len(rows)], b[len(rows):]
    out = []
    for k in range(len(rows)):
        out.append((model["col"][lo[k]:hi[k]].cpu().numpy(), model["cnt"][lo[k]:hi[k]].cpu().numpy().astype(np.int64)))
    return out


@pytest.mark.parametrize("which", ["paper_shaped", "large"])
def test_full_size_sampled(planner, ora, which):
    from paper_2109_00857_amd import mdp

    w = W.config2() if which == "paper_shaped" else W.config3()
    p = w.problem
    nx, ny, nt, nr = p["nx"], p["ny"], p["nt"], p["n_real"]
    nc, na = nx * ny, w.n_actions
    ns = w.n_states
    print(f"[full] {which}: {nx}x{ny}x{nt}, Nr={nr}, Na={na}, rows={w.n_rows}", flush=True)
    env = planner.upload_env(w)
    mdp.mdp_autotune(planner.ctx, p, env)
    model, st = planner.build(p, env)
    mdp.mdp_ctx_set_plan(planner.ctx, p, 0, 0, 0)
    assert st["status"] == 0 and st["n_escape"] == 0, st
    print(f"[full] {which}: nnz={st['nnz']}", flush=True)
    missions = w.missions()
    rng = np.random.default_rng(2024)

    # ---- sampled rows, plus the rows on each side of the build passes' layer
    # boundaries (the large instance is built 8 layers per pass)
    edges = [b * nc * na + d for b in range(8, nt, 8) for d in (-1, 0)]
    rows = np.unique(np.concatenate([rng.choice(w.n_rows, N_ROWS, replace=False), edges]))
    got = _rows_of(model, rows)
    import torch

    Rg = model["reward"][:, torch.as_tensor(rows, device=model["reward"].device)].cpu().numpy().astype(np.float64)
    for k, row in enumerate(rows):
        s, a = divmod(int(row), na)
        t, c = divmod(s, nc)
        cols, cnts, R, A, ne, _ = ora.row(w, t, c, a)
        assert ne == 0
        np.testing.assert_array_equal(got[k][0], cols, err_msg=f"row {row}")
        np.testing.assert_array_equal(got[k][1], cnts, err_msg=f"row {row}")
        for slot, m in enumerate(missions):
            assert abs(Rg[slot, k] - R[m]) <= 1e-5 * A[m], (row, m, Rg[slot, k], R[m], A[m])

    # ---- sampled states: Bellman identity and greedy optimality
    states = rng.choice(ns, N_STATES, replace=False)
    oracle_rows = {}
    for s in states:
        t, c = divmod(int(s), nc)
        oracle_rows[int(s)] = [ora.row(w, t, c, a) for a in range(na)]
    # the missions solved together, as the benchmark step does
    vs, vsts = planner.value_iterate_missions(p, model, missions)
    if which == "paper_shaped":  # against the oracle's exact solution at its sampled states
        with open(os.path.join(GOLDEN, "paper_shaped_values.json")) as f:
            g = json.load(f)
        assert g["nnz"] == st["nnz"]
        gs = np.array(g["states"])
        for m, v in zip(missions, vs):
            o = g["missions"][str(m)]
            vg = v.cpu().numpy()[gs]
            v_o, w_o, q_o = np.array(o["v"]), np.array(o["w"]), np.array(o["q"])
            err = np.abs(vg - v_o)
            assert np.all(err <= REL_TOL * w_o), (m, gs[err > REL_TOL * w_o][:5])
            pi = planner.policy(p, model, m, v).cpu().numpy()[gs]
            qa = q_o[np.arange(len(gs)), pi]
            assert np.all(qa >= q_o.max(axis=1) - REL_TOL * w_o), m
            print(f"[full] paper_shaped mission {m}: {len(gs)} states against the oracle's solution, "
                  f"worst |dv|/w = {float(np.max(err / np.maximum(w_o, 1e-300))):.2e}", flush=True)
    for m, v, vst in zip(missions, vs, vsts):
        assert vst["status"] == 0 and vst["sweeps"] <= nt + 1, vst
        pi = planner.policy(p, model, m, v).cpu().numpy()
        v = v.cpu().numpy()
        worst = 0.0
        for s in states:
            q = np.zeros(na)
            scale = 0.0
            for a, (cols, cnts, R, A, _, _) in enumerate(oracle_rows[int(s)]):
                trans = cols < ns
                ev = float((cnts[trans] * v[cols[trans]]).sum()) / nr
                eabs = float((cnts[trans] * np.abs(v[cols[trans]])).sum()) / nr
                q[a] = R[m] + ev
                scale = max(scale, A[m] + eabs)
            tol = 1e-5 * scale
            assert abs(v[s] - q.max()) <= tol, (which, m, int(s), v[s], q.max(), scale)
            assert q[pi[s]] >= q.max() - tol, (which, m, int(s), pi[s], q[pi[s]], q.max())
            if scale > 0:
                worst = max(worst, abs(v[s] - q.max()) / scale)
        print(f"[full] {which} mission {m}: sweeps={vst['sweeps']} worst rel Bellman gap={worst:.2e}", flush=True)
        # the GPU policy rolled out in every realization, on the GPU and in the oracle
        traj, paths, rst = planner.rollout(p, env, torch.from_numpy(pi).to(planner.device))
        ro = ora.rollout(w, pi)
        np.testing.assert_array_equal(traj.cpu().numpy().T, ro["traj"])
        np.testing.assert_array_equal(paths["outcome"], ro["outcome"])
        assert np.allclose(paths["ret"], ro["ret"], rtol=1e-12, atol=1e-9)
        assert rst["n_arrived"] == ro["n_arrived"]
        print(f"[full] {which} mission {m}: rollouts P(reach)={rst['p_reach']:.4f} "
              f"E[time|arrived]={rst['mean_time_arrived']:.4g}", flush=True)
