"""Pins of the oracle's swept-path obstacle test (the reading of Alg. 2's
"obstacle between s and s'" in which the straight path of the step must not
enter an obstacle cell at t+1): the segment-cell test against Liang-Barsky
clipping, hand-built crossings, and the model against an independent
double-precision evaluation."""
import numpy as np
import pytest

from paper_2109_00857_amd import workloads as W


def _liang_barsky_meets_open(x0, y0, x1, y1, a, b):
    """Clip the segment to the closed square [a, a+1] x [b, b+1] (Liang-Barsky);
    it meets the open square iff the clipped part has positive length and its
    midpoint lies strictly inside."""
    dx, dy = x1 - x0, y1 - y0
    t0, t1 = 0.0, 1.0
    for p, q in ((-dx, x0 - a), (dx, a + 1 - x0), (-dy, y0 - b), (dy, b + 1 - y0)):
        if p == 0:
            if q < 0:
                return False
        else:
            r = q / p
            if p < 0:
                t0 = max(t0, r)
            else:
                t1 = min(t1, r)
    if t1 <= t0:
        return False
    tm = 0.5 * (t0 + t1)
    xm, ym = x0 + tm * dx, y0 + tm * dy
    return a < xm < a + 1 and b < ym < b + 1


def test_segment_cell_hand_cases(ora):
    f = ora.segment_meets_cell
    assert f(0.5, 0.5, 2.5, 0.5, 1, 0) and f(0.5, 0.5, 2.5, 0.5, 2, 0) and not f(0.5, 0.5, 2.5, 0.5, 1, 1)
    # through the corner (1, 1): the diagonal neighbours are touched at a point only
    assert f(0.5, 0.5, 1.5, 1.5, 1, 1) and not f(0.5, 0.5, 1.5, 1.5, 1, 0) and not f(0.5, 0.5, 1.5, 1.5, 0, 1)
    # ending exactly on an edge: the cell beyond it is not entered
    assert not f(0.5, 0.5, 1.0, 0.5, 1, 0) and f(0.5, 0.5, 1.0 + 2 ** -20, 0.5, 1, 0)
    # a degenerate segment enters nothing
    assert not f(0.5, 0.5, 0.5, 0.5, 0, 0)
    # a shallow segment that clips the corner region of a neighbour
    assert f(0.5, 0.5, 3.5, 1.2, 2, 1) and not f(0.5, 0.5, 3.5, 1.2, 1, 1)


def test_segment_cell_against_clipping(ora):
    rng = np.random.default_rng(8)
    n = 0
    for _ in range(3000):
        i, j = rng.integers(0, 6, 2)
        x0, y0 = i + 0.5, j + 0.5
        # fp32 landing coordinates, some snapped to edges or to the centre lines
        x1, y1 = (np.float32(x0 + rng.uniform(-3, 3)), np.float32(y0 + rng.uniform(-3, 3)))
        if rng.random() < 0.2:
            x1 = np.float32(np.round(x1))
        if rng.random() < 0.2:
            y1 = np.float32(y0 + rng.integers(-2, 3))
        x1, y1 = float(x1), float(y1)
        for a in range(int(np.floor(min(x0, x1))) - 1, int(np.floor(max(x0, x1))) + 2):
            for b in range(int(np.floor(min(y0, y1))) - 1, int(np.floor(max(y0, y1))) + 2):
                assert ora.segment_meets_cell(x0, y0, x1, y1, a, b) == _liang_barsky_meets_open(x0, y0, x1, y1, a, b), \
                    (x0, y0, x1, y1, a, b)
                n += 1
    assert n > 20000


def test_swept_path_jumps_over_an_obstacle(ora):
    """A fast step of two cells east from (1, 2) lands in (3, 2); an obstacle at
    (2, 2) at t+1 lies on its path: DEAD with the swept test, a free landing
    without it; an obstacle beside the path changes nothing."""
    w = W.uniform_flow(6, 5, 3, 0.0, 0.0, n_real=4, n_head=4, f_max=1.6, start=(0, 0), target=(5, 4), sub_h=2,
                       n_speed=2)
    ns = 3 * 30
    c = 2 * 6 + 1
    fast_east = 4  # speed 1 (fast), heading 0
    cols, _, R, _, _, _ = ora.row(w, 0, c, fast_east)
    assert list(cols) == [30 + 2 * 6 + 3]
    mask = np.zeros((4, 5, 6), np.uint8)
    mask[1, 2, 2] = 1
    w.mask = mask
    cols, _, _, _, _, _ = ora.row(w, 0, c, fast_east)
    assert list(cols) == [30 + 2 * 6 + 3]  # the landing rule alone does not see it
    w.problem["flags"] |= ora.FLAG_SWEPT_PATH
    cols, _, R, _, _, _ = ora.row(w, 0, c, fast_east)
    assert list(cols) == [ns] and R[0] == -1000.0
    mask[1, 2, 2] = 0
    mask[1, 3, 2] = 1  # beside the path
    cols, _, _, _, _, _ = ora.row(w, 0, c, fast_east)
    assert list(cols) == [30 + 2 * 6 + 3]
    mask[0, 2, 2] = 1  # an obstacle at t only, not t+1: the path is free
    mask[1, 3, 2] = 0
    cols, _, _, _, _, _ = ora.row(w, 0, c, fast_east)
    assert list(cols) == [30 + 2 * 6 + 3]


def test_swept_model_against_fp64(ora):
    """Stochastic flow with moving discs, two speeds: with the swept test, each
    row's counts equal an independent fp64 evaluation (physical landing, then
    the segment against the obstacles at t+1 by Liang-Barsky clipping) on rows
    without near-edge samples, and only ever move samples into DEAD."""
    w = W.config2(nx=22, ny=20, nt=3, n_real=60, K=4, n_head=8)
    w.problem["n_speed"] = 2
    w.problem["f_max"] = 0.9
    w.problem["sub_hx"] = w.problem["sub_hy"] = 4
    m0 = ora.build_model(w)
    w.problem["flags"] |= ora.FLAG_SWEPT_PATH
    m1 = ora.build_model(w)
    p = w.problem
    nx, ny, nt, K = p["nx"], p["ny"], p["nt"], p["n_modes"]
    nc, na, ns = nx * ny, w.n_actions, w.n_states
    assert m0["n_escape"] == 0
    moved = 0
    checked = 0
    for t in range(nt):
        mu = w.mu[t].astype(np.float64)
        u = w.ubar[0].reshape(-1, 1).astype(np.float64) + np.einsum("kc,kr->cr", w.phiu[0].reshape(K, -1), mu)
        v = w.vbar[0].reshape(-1, 1).astype(np.float64) + np.einsum("kc,kr->cr", w.phiv[0].reshape(K, -1), mu)
        for a in range(na):
            h, jf = a % p["n_head"], a // p["n_head"]
            F = p["f_max"] * (jf + 1) / p["n_speed"]
            th = 2 * np.pi * h / p["n_head"]
            for c in range(nc):
                row = (t * nc + c) * na + a
                i, j = c % nx, c // nx
                if (i, j) == (p["target_i"], p["target_j"]) or w.mask[t, j, i]:
                    continue
                lo0, hi0 = m0["row_ptr"][row], m0["row_ptr"][row + 1]
                lo1, hi1 = m1["row_ptr"][row], m1["row_ptr"][row + 1]
                d0 = dict(zip(m0["col"][lo0:hi0].tolist(), m0["cnt"][lo0:hi0].tolist()))
                d1 = dict(zip(m1["col"][lo1:hi1].tolist(), m1["cnt"][lo1:hi1].tolist()))
                for col, n in d1.items():  # only moves into DEAD
                    assert col == ns or n <= d0.get(col, 0)
                moved += d1.get(ns, 0) - d0.get(ns, 0)
                if m0["row_near"][row]:
                    continue
                X = (i + 0.5) + (u[c] + F * np.cos(th)) * p["dt"] / p["dx"]
                Y = (j + 0.5) + (v[c] + F * np.sin(th)) * p["dt"] / p["dy"]
                exp = {}
                for x1, y1 in zip(X, Y):
                    ip, jp = int(np.floor(x1)), int(np.floor(y1))
                    if not (0 <= ip < nx and 0 <= jp < ny) or w.mask[t + 1, jp, ip]:
                        col = ns
                    else:
                        blocked = any(w.mask[t + 1, b, a2] and (a2, b) != (i, j) and
                                      _liang_barsky_meets_open(i + 0.5, j + 0.5, x1, y1, a2, b)
                                      for a2 in range(max(0, min(i, ip)), min(nx, max(i, ip) + 1))
                                      for b in range(max(0, min(j, jp)), min(ny, max(j, jp) + 1)))
                        if blocked:
                            col = ns
                        elif (ip, jp) == (p["target_i"], p["target_j"]):
                            col = ns + 1
                        elif t + 1 == nt:
                            col = ns
                        else:
                            col = (t + 1) * nc + jp * nx + ip
                    exp[col] = exp.get(col, 0) + 1
                assert exp == d1, (t, c, a)
                checked += 1
    assert moved > 0 and checked > 5000
