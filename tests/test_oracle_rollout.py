"""Pins of the oracle's policy rollouts through the realization ensemble
(Sec. IV: each optimal policy applied to every flow realization): the
hand-derived worked example, deterministic flows whose realized return is the
optimal value, and an independent double-precision re-simulation of every path
in physical units."""
import json
import math
import os

import numpy as np
import pytest

from paper_2109_00857_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _a1(nt):
    with open(os.path.join(GOLDEN, "worked_example_uniform_flow.json")) as f:
        g = json.load(f)["setup"]
    return W.uniform_flow(g["nx"], g["ny"], nt, g["u0"], g["v0"], n_real=5, n_head=g["n_head"], f_max=g["f_max"],
                          dx=g["dx"], dy=g["dy"], dt=g["dt"], start=tuple(g["start"]), target=tuple(g["target"]),
                          sub_h=2)


def test_rollout_worked_example(ora):
    """Deterministic uniform flow (hand-derived): with T = 3 every realization goes
    E, E, E and arrives after 3 steps with return 97; with T = 2 every path ends
    beyond the horizon with return -1001 (the optimal values at the start)."""
    w = _a1(3)
    m = ora.build_model(w)
    _, pi, _ = ora.backward(w, m, 0)
    ro = ora.rollout(w, pi)
    nx = w.problem["nx"]
    assert (ro["outcome"] == ora.ROLL_ARRIVED).all() and (ro["steps"] == 3).all()
    assert (ro["traj"] == np.array([1 * nx + 0, 1 * nx + 1, 1 * nx + 2, 1 * nx + 3])).all()
    assert (ro["ret"][:, 0] == 97.0).all()
    assert ro["p_reach"] == 1.0 and ro["mean_time_arrived"] == 3.0
    w2 = _a1(2)
    m2 = ora.build_model(w2)
    _, pi2, _ = ora.backward(w2, m2, 0)
    ro2 = ora.rollout(w2, pi2)
    assert (ro2["outcome"] == ora.ROLL_HORIZON).all() and (ro2["ret"][:, 0] == -1001.0).all()
    assert (ro2["traj"][:, 2] == -1).all() and ro2["p_reach"] == 0.0


@pytest.mark.parametrize("mission", [0, 1, 2])
def test_rollout_deterministic_return_is_optimal_value(ora, mission):
    """With every coefficient zero the flow is deterministic: every realization
    follows the same path and its realized return is the optimal value at the
    start; energy is c_f F^2 dt per step."""
    w = W.config2(nx=20, ny=22, nt=14, n_real=6, K=4, n_head=8)
    w.mu[:] = 0.0
    w.problem["n_speed"] = 2
    m = ora.build_model(w)
    v, pi, _ = ora.backward(w, m, mission)
    ro = ora.rollout(w, pi)
    p = w.problem
    s0 = p["start_j"] * p["nx"] + p["start_i"]
    assert (ro["traj"] == ro["traj"][0]).all()
    assert np.allclose(ro["ret"][:, mission], v[s0], rtol=1e-12, atol=1e-9), (ro["ret"][0], v[s0])
    # energy and speed along the path from the actions taken
    t, c, e, f = 0, s0, 0.0, 0.0
    nc = p["nx"] * p["ny"]
    for t in range(ro["steps"][0]):
        c = ro["traj"][0, t]
        a = pi[t * nc + c]
        F = p["f_max"] * (a // p["n_head"] + 1) / p["n_speed"]
        e += p["c_f"] * F * F * p["dt"]
        f += F
    assert abs(ro["energy"][0] - e) <= 1e-12 * e and abs(ro["fsum"][0] - f) <= 1e-12 * f


def _fp64_rollout(w, pi):
    """Independent re-simulation in double precision and physical units: position
    (i + 1/2) dx + (u_r(t, cell) + F_a cos th_a) dt with u_r = ubar + sum_k mu_k(t, r)
    phi_k, cell() = floor, the landing rules of the model; returns trajectories,
    outcomes, steps, returns, and per step the distance (cell units) of the
    landing from the nearest cell edge."""
    p = w.problem
    nx, ny, nt, nr, K = p["nx"], p["ny"], p["nt"], p["n_real"], p["n_modes"]
    nc = nx * ny
    dx, dy, dt = p["dx"], p["dy"], p["dt"]
    nh = p["n_head"]
    traj = -np.ones((nr, nt + 1), np.int64)
    out = np.full(nr, 3, np.int64)
    steps = np.zeros(nr, np.int64)
    ret = np.zeros((nr, 3))
    edge = np.full((nr, nt), np.inf)
    i = np.full(nr, p["start_i"])
    j = np.full(nr, p["start_j"])
    alive = np.ones(nr, bool)
    traj[:, 0] = j * nx + i
    g = w.gbar if w.gbar is not None else np.zeros((nt + 1, ny, nx), np.float32)
    for t in range(nt):
        rs = np.flatnonzero(alive)
        if len(rs) == 0:
            break
        c = j[rs] * nx + i[rs]
        tgt = (i[rs] == p["target_i"]) & (j[rs] == p["target_j"])
        out[rs[tgt]] = 0
        alive[rs[tgt]] = False
        rs, c = rs[~tgt], c[~tgt]
        if w.mask is not None:
            ob = w.mask[t].reshape(-1)[c].astype(bool)
            ret[rs[ob]] += p["r_outbound"]
            out[rs[ob]] = 2
            alive[rs[ob]] = False
            rs, c = rs[~ob], c[~ob]
        tm = t if p["mean_time_varying"] else 0
        tp = t if p["mode_time_varying"] else 0
        mu = w.mu[t][:, rs].astype(np.float64)  # [K][n]
        u = w.ubar[tm].reshape(-1)[c].astype(np.float64) + (w.phiu[tp].reshape(K, -1)[:, c] * mu).sum(0)
        v = w.vbar[tm].reshape(-1)[c].astype(np.float64) + (w.phiv[tp].reshape(K, -1)[:, c] * mu).sum(0)
        a = pi[t * nc + c]
        F = p["f_max"] * (a // nh + 1) / p["n_speed"]
        th = 2.0 * math.pi * (a % nh) / nh
        X = ((c % nx) + 0.5) + (u + F * np.cos(th)) * dt / dx
        Y = ((c // nx) + 0.5) + (v + F * np.sin(th)) * dt / dy
        edge[rs, t] = np.minimum(np.abs(X - np.round(X)), np.abs(Y - np.round(Y)))
        ip, jp = np.floor(X).astype(np.int64), np.floor(Y).astype(np.int64)
        steps[rs] += 1
        e_a = p["c_f"] * F * F
        inside = (ip >= 0) & (ip < nx) & (jp >= 0) & (jp < ny)
        cp = np.where(inside, jp * nx + ip, 0)
        blocked = inside & (w.mask[t + 1].reshape(-1)[cp].astype(bool) if w.mask is not None else False)
        dead = ~inside | blocked
        ret[rs[dead]] += p["r_outbound"]
        out[rs[~inside]] = 1
        out[rs[blocked]] = 2
        base = np.stack([-dt + 0 * F, -e_a * dt,
                         (-e_a + 0.5 * p["c_r"] * g[t].reshape(-1)[c] + 0.5 * p["c_r"] * g[t + 1].reshape(-1)[cp]) * dt], 1)
        arrive = ~dead & (ip == p["target_i"]) & (jp == p["target_j"])
        ret[rs[arrive]] += base[arrive] + p["r_term"]
        out[rs[arrive]] = 0
        horizon = ~dead & ~arrive & (t + 1 == nt)
        ret[rs[horizon]] += p["r_outbound"]
        go = ~dead & ~arrive & ~horizon
        ret[rs[go]] += base[go]
        traj[rs[arrive | go], t + 1] = cp[arrive | go]
        alive[rs[~go]] = False
        i[rs[go]] = ip[go]
        j[rs[go]] = jp[go]
    return traj, out, steps, ret, edge


@pytest.mark.parametrize("mission", [0, 1, 2])
def test_rollout_matches_fp64_physics(ora, mission):
    """Stochastic AR(1) flow, obstacles, two speeds: every path whose landings all
    stay clear of cell edges in the fp64 re-simulation has the oracle's
    trajectory, outcome and step count exactly and its returns within 1e-12; the
    others first differ at a landing within 1e-4 cells of an edge."""
    w = W.config1(nx=16, ny=16, nt=14, n_real=300, n_head=8, sub_h=4)
    p = w.problem
    p.update(n_speed=2, f_max=0.8, start_i=2, start_j=2, target_i=10, target_j=10, mission_mask=7)
    w.gbar = W._gaussian_bump(16, 16, 14)
    m = ora.build_model(w)
    assert m["n_escape"] == 0
    _, pi, _ = ora.backward(w, m, mission)
    ro = ora.rollout(w, pi)
    traj, out, steps, ret, edge = _fp64_rollout(w, pi)
    clear = (edge >= 1e-4).all(axis=1)
    assert clear.mean() > 0.98
    np.testing.assert_array_equal(ro["traj"][clear], traj[clear])
    np.testing.assert_array_equal(ro["outcome"][clear], out[clear])
    np.testing.assert_array_equal(ro["steps"][clear], steps[clear])
    assert np.allclose(ro["ret"][clear], ret[clear], rtol=1e-12, atol=1e-9)
    for r in np.flatnonzero(~clear):
        if not np.array_equal(ro["traj"][r], traj[r]):
            k = int(np.flatnonzero(ro["traj"][r] != traj[r])[0])
            assert edge[r, k - 1] < 1e-4, (r, k)
    assert ro["p_reach"] > 0.1 and len(set(ro["outcome"].tolist())) >= 2


def test_rollout_first_step_is_the_policy_row(ora):
    """Across the ensemble, the first landings from the start are distributed
    exactly as the model's row (0, start, pi(0, start)): same samples, same rules."""
    w = W.config2(nx=24, ny=22, nt=4, n_real=2000, K=6, n_head=12)
    m = ora.build_model(w)
    _, pi, _ = ora.backward(w, m, 2)
    ro = ora.rollout(w, pi)
    p = w.problem
    nc = p["nx"] * p["ny"]
    ns = w.n_states
    s0 = p["start_j"] * p["nx"] + p["start_i"]
    row = s0 * w.n_actions + pi[s0]
    lo, hi = m["row_ptr"][row], m["row_ptr"][row + 1]
    exp = dict(zip(m["col"][lo:hi].tolist(), m["cnt"][lo:hi].tolist()))
    got = {}
    for r in range(p["n_real"]):
        if ro["steps"][r] == 0:
            continue
        if ro["traj"][r, 1] >= 0:
            col = nc + ro["traj"][r, 1] if ro["traj"][r, 1] != p["target_j"] * p["nx"] + p["target_i"] else ns + 1
        else:
            col = ns
        got[col] = got.get(col, 0) + 1
    assert got == exp
