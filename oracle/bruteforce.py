"""Exhaustive policy search on tiny grids: TEST INFRASTRUCTURE ONLY.

An optimal deterministic Markov policy exists for the finite-horizon,
undiscounted, total-cost MDP (Sec. II-B). On a tiny grid every such policy
restricted to the states reachable from the start can be enumerated and
evaluated by pushing the start distribution forward through the transition
probabilities; the best expected return must equal the optimal value at the
start. This is independent of the backward-induction code in mdp_oracle.c.
"""
from __future__ import annotations

import numpy as np


def reachable_layers(model: dict, problem: dict, n_actions: int):
    """States reachable from the start, layer by layer (sinks excluded)."""
    nx, ny, nt = problem["nx"], problem["ny"], problem["nt"]
    nc = nx * ny
    ns = nt * nc
    s0 = problem["start_j"] * nx + problem["start_i"]
    layers = [[s0]]
    rp, col = model["row_ptr"], model["col"]
    for t in range(nt - 1):
        nxt = set()
        for s in layers[-1]:
            for a in range(n_actions):
                r = s * n_actions + a
                for k in range(rp[r], rp[r + 1]):
                    if col[k] < ns:
                        nxt.add(int(col[k]))
        layers.append(sorted(nxt))
    return layers


def best_policy_return(model: dict, problem: dict, mission: int, max_policies: int = 1 << 22):
    """Maximum over all deterministic Markov policies of the expected total reward
    from the start state. Returns (best_return, n_policies)."""
    na = problem["n_head"] * problem["n_speed"]
    nr = problem["n_real"]
    nx, ny, nt = problem["nx"], problem["ny"], problem["nt"]
    ns = nt * nx * ny
    layers = reachable_layers(model, problem, na)
    states = [s for layer in layers for s in layer]
    n_pol = na ** len(states)
    if n_pol > max_policies:
        raise ValueError(f"{n_pol} policies is too many for exhaustive search")
    pol = np.arange(n_pol, dtype=np.int64)
    digit = {s: (pol // (na ** k)) % na for k, s in enumerate(states)}
    R = model["R"][mission]
    rp, col, cnt = model["row_ptr"], model["col"], model["cnt"]

    prob = {layers[0][0]: np.ones(n_pol)}
    total = np.zeros(n_pol)
    for layer in layers:
        for s in layer:
            q = prob.pop(s, None)
            if q is None:
                continue
            a_s = digit[s]
            rew = np.array([R[s * na + a] for a in range(na)])
            total += q * rew[a_s]
            for a in range(na):
                sel = a_s == a
                if not sel.any():
                    continue
                r = s * na + a
                for k in range(rp[r], rp[r + 1]):
                    c = int(col[k])
                    if c < ns:
                        prob.setdefault(c, np.zeros(n_pol))
                        prob[c] += np.where(sel, q * (cnt[k] / nr), 0.0)
    return float(total.max()), n_pol
