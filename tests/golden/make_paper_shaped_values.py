"""Writes tests/golden/paper_shaped_values.json: the CPU oracle's exact solution
of the full-size paper-shaped instance (100 x 100 cells, 120 layers, 10 modes,
5000 AR(1) realizations, 16 headings, 5 x 5 sub-grid, three missions) at 100
sampled states: for each mission the backward-induction value v (Sec. II-B
Bellman equation over the layered model of Sec. II-A and Alg. 2), the value of
the absolute rewards under the oracle's policy (the tolerance scale) and Q of
every action.

Calls only oracle/ and the seeded input generator. The model is built in layer
ranges on several processes (the oracle is single-threaded) and joined; about
90 CPU-minutes in all.

    python tests/golden/make_paper_shaped_values.py [--procs 8]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2109_00857_amd import workloads as W  # noqa: E402

N_STATES = 100
SEED = 31
OUT = os.path.join(HERE, "paper_shaped_values.json")


def _part(rng_):
    t0, t1 = rng_
    return oracle.build_layers(W.config2(), t0, t1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    args = ap.parse_args()
    w = W.config2()
    nt = w.problem["nt"]
    ranges = [(t, min(t + 4, nt)) for t in range(0, nt, 4)]
    t_start = time.time()
    with Pool(args.procs) as pool:
        parts = []
        for k, part in enumerate(pool.imap(_part, ranges)):
            parts.append(part)
            print(f"layers {ranges[k][0]}..{ranges[k][1] - 1} built ({time.time() - t_start:.0f} s)", flush=True)
    model = oracle.concat_layers(parts)
    del parts
    assert model["n_escape"] == 0
    states = np.sort(np.random.default_rng(SEED).choice(w.n_states, N_STATES, replace=False))
    out = dict(
        citation="The oracle's backward induction (Sec. II-B) on its own model of the paper-shaped instance "
                 "(Sec. II-A transitions and rewards, Alg. 2), written by tests/golden/make_paper_shaped_values.py",
        workload="config2(): 100x100 cells, 120 layers, 10 modes, 5000 AR(1) realizations, 16 headings, 5x5 "
                 "sub-grid, 4 moving discs, time / energy / net-energy missions, seed 0",
        nnz=model["nnz"], states=[int(s) for s in states], missions={})
    for m in w.missions():
        v, pi, wabs = oracle.backward(w, model, m)
        q = oracle.q_values(w, model, m, v, states)
        out["missions"][str(m)] = dict(v=[float(v[s]) for s in states], w=[float(wabs[s]) for s in states],
                                       q=[[float(x) for x in row] for row in q])
        print(f"mission {m}: v(start layer) in [{v[:10000].min():.6g}, {v[:10000].max():.6g}]", flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {OUT} ({time.time() - t_start:.0f} s)")


if __name__ == "__main__":
    main()
