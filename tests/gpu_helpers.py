"""Shared checks for the GPU parity tests: the HIP path against the CPU oracle."""
from __future__ import annotations

import numpy as np

# Values and rewards agree within 1e-5 of the oracle's absolute-reward scale
# (expected |reward| of the row for R; the value of |rewards| under the oracle's
# policy for v).
REL_TOL = 1e-5


def model_to_host(model: dict, stats: dict) -> dict:
    nnz = stats["nnz"]
    return dict(
        row_ptr=model["row_ptr"].cpu().numpy(),
        col=model["col"][:nnz].cpu().numpy(),
        cnt=model["cnt"][:nnz].cpu().numpy().astype(np.int32),
        reward=model["reward"].cpu().numpy(),
    )


def assert_counts_equal(g: dict, o: dict) -> None:
    """Transition counts bit-exact: row pointers, columns and counts."""
    np.testing.assert_array_equal(g["row_ptr"], o["row_ptr"])
    np.testing.assert_array_equal(g["col"], o["col"])
    np.testing.assert_array_equal(g["cnt"], o["cnt"])


def assert_rewards_close(g: dict, o: dict, missions: list[int]) -> float:
    """|R_gpu - R_oracle| <= 1e-5 * E|r| per row (exactly equal when E|r| = 0)."""
    worst = 0.0
    for slot, m in enumerate(missions):
        Rg = g["reward"][slot].astype(np.float64)
        Ro = o["R"][m]
        A = o["A"][m]
        err = np.abs(Rg - Ro)
        bad = err > REL_TOL * A
        assert not bad.any(), (m, np.flatnonzero(bad)[:10], Rg[bad][:5], Ro[bad][:5], A[bad][:5])
        with np.errstate(divide="ignore", invalid="ignore"):
            r = np.where(A > 0, err / A, 0.0)
        worst = max(worst, float(r.max(initial=0.0)))
    return worst


def assert_values_close(v_gpu: np.ndarray, v_ora: np.ndarray, w_ora: np.ndarray) -> float:
    err = np.abs(v_gpu - v_ora)
    bad = err > REL_TOL * w_ora
    assert not bad.any(), (np.flatnonzero(bad)[:10], v_gpu[bad][:5], v_ora[bad][:5], w_ora[bad][:5])
    with np.errstate(divide="ignore", invalid="ignore"):
        return float(np.where(w_ora > 0, err / w_ora, 0.0).max(initial=0.0))


def assert_policy_optimal(ora, w, om: dict, mission: int, v_ora, w_ora, pi_gpu) -> float:
    """The GPU's action attains the oracle's max Q within the value tolerance.
    Returns the exact-match rate with the oracle's policy."""
    ns = w.n_states
    q = ora.q_values(w, om, mission, v_ora, np.arange(ns))
    qmax = q.max(axis=1)
    qg = q[np.arange(ns), pi_gpu]
    bad = qg < qmax - REL_TOL * w_ora
    assert not bad.any(), (np.flatnonzero(bad)[:10], qg[bad][:5], qmax[bad][:5])
    _, pi_ora, _ = ora.backward(w, om, mission)
    return float((pi_ora == pi_gpu).mean())


def assert_matches_oracle(ora, w, missions, g: dict, stats: dict, values: dict, policies: dict,
                          om: dict | None = None) -> dict:
    """Whole-model parity of one problem's GPU outputs against the oracle:
    counts bit-exact, rewards within tolerance, and for each solved mission the
    values within tolerance and the policy optimal within it.
    g: model_to_host(...) of the GPU model (reward slots in ascending mission
    order of w's mission mask); values / policies: mission -> numpy array."""
    if om is None:
        om = ora.build_model(w)
    assert stats["nnz"] == om["nnz"], (stats["nnz"], om["nnz"])
    assert stats["n_escape"] == om["n_escape"] == 0
    if stats.get("n_near_edge", -1) >= 0:
        assert stats["n_near_edge"] == om["n_near_edge"]
    assert_counts_equal(g, om)
    assert_rewards_close(g, om, w.missions())
    for m in missions:
        v_ora, _, w_ora = ora.backward(w, om, m)
        assert_values_close(values[m], v_ora, w_ora)
        assert_policy_optimal(ora, w, om, m, v_ora, w_ora, policies[m])
    return om





def landing_loop(problem: dict) -> str:
    """The landing loop the library takes for a 16-bit-counter build of `problem`,
    by the same rule as its host code: "pairs" when N_a is even and some two
    actions have bitwise-equal fp32 x displacements (each evaluated in double
    and rounded once, axis headings exact), else "rows" (one lane per row).
    Used to check that the tests cover both loops."""
    import math

    nh, ns = problem["n_head"], problem["n_speed"]
    na = nh * ns
    if na < 2 or na % 2:
        return "rows"
    axis_x = {0: 1.0, 1: 0.0, 2: -1.0, 3: 0.0}
    hx = []
    for jf in range(ns):
        F = problem["f_max"] * (jf + 1) / ns
        for h in range(nh):
            c = axis_x[4 * h // nh] if (4 * h) % nh == 0 else math.cos(2.0 * math.pi * h / nh)
            hx.append(np.float32(F * c * problem["dt"] / problem["dx"]).tobytes())
    return "pairs" if len(set(hx)) < na else "rows"
