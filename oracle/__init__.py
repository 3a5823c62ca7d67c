"""CPU oracle of the stochastic-flow MDP planner: TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct reference of the planner's results, written
from the paper (Sec. II-A transition model and rewards, Sec. II-B Bellman
equation and value iteration, Sec. II-C reduced-order flow, Sec. III-A mean
scalar-field result). The arithmetic lives in ``mdp_oracle.c`` (plain C,
compiled with gcc ``-O2 -ffp-contract=off``); this module only builds and
marshals it, plus a pure-Python exhaustive policy search for tiny grids
(``bruteforce.py``).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package. It shares no code with the GPU planner.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mdp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so."""
    cmd = ["gcc", *CFLAGS, "-o", _LIB + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class OraProblem(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nt", C.c_int32),
        ("n_modes", C.c_int32), ("n_real", C.c_int32),
        ("n_head", C.c_int32), ("n_speed", C.c_int32),
        ("sub_hx", C.c_int32), ("sub_hy", C.c_int32),
        ("start_i", C.c_int32), ("start_j", C.c_int32),
        ("target_i", C.c_int32), ("target_j", C.c_int32),
        ("mean_time_varying", C.c_int32), ("mode_time_varying", C.c_int32),
        ("mission_mask", C.c_uint32), ("flags", C.c_uint32),
        ("dx", C.c_double), ("dy", C.c_double), ("dt", C.c_double), ("f_max", C.c_double),
        ("r_term", C.c_double), ("r_outbound", C.c_double), ("c_f", C.c_double), ("c_r", C.c_double),
    ]


class OraEnv(C.Structure):
    _fields_ = [
        ("ubar", C.c_void_p), ("vbar", C.c_void_p),
        ("phiu", C.c_void_p), ("phiv", C.c_void_p),
        ("mu", C.c_void_p), ("gbar", C.c_void_p), ("mask", C.c_void_p),
    ]


_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = C.CDLL(_LIB)
        P, E = C.POINTER(OraProblem), C.POINTER(OraEnv)
        vp = C.c_void_p
        lib.ora_action_tables.argtypes = [P, vp, vp, vp]
        lib.ora_landing.argtypes = [P, E, C.c_int, C.c_int, C.c_int, C.c_int, vp, vp, vp]
        lib.ora_row.argtypes = [P, E, C.c_int, C.c_int, C.c_int, vp, vp, vp, vp, vp, vp]
        lib.ora_row.restype = C.c_int32
        lib.ora_build.argtypes = [P, E, vp, vp, vp, C.c_int64, vp, vp, vp, vp, vp]
        lib.ora_build.restype = C.c_int64
        lib.ora_build_layers.argtypes = [P, E, C.c_int, C.c_int, vp, vp, vp, C.c_int64, vp, vp, vp, vp, vp]
        lib.ora_build_layers.restype = C.c_int64
        lib.ora_backward.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.ora_jacobi.argtypes = [P, vp, vp, vp, vp, C.c_double, C.c_int32, vp, vp]
        lib.ora_jacobi.restype = C.c_int32
        lib.ora_q.argtypes = [P, vp, vp, vp, vp, vp, vp, C.c_int64, vp]
        lib.ora_rollout.argtypes = [P, E, vp, vp, vp, vp, vp, vp, vp]
        lib.ora_segment_meets_cell.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, C.c_int]
        lib.ora_segment_meets_cell.restype = C.c_int
        lib.ora_max_speed.argtypes = [P, E, vp, vp]
        lib.ora_subgrid_auto.argtypes = [P, E, vp, vp]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def problem_struct(p: dict) -> OraProblem:
    return OraProblem(**{k: p[k] for k, _ in OraProblem._fields_})


class _Bound:
    """Keeps the numpy arrays alive while C holds raw pointers to them."""

    def __init__(self, w):
        self.p = problem_struct(w.problem)
        self.arrays = [np.ascontiguousarray(x) if x is not None else None
                       for x in (w.ubar, w.vbar, w.phiu, w.phiv, w.mu, w.gbar, w.mask)]
        self.e = OraEnv(*[_ptr(a) for a in self.arrays])


def n_actions(w) -> int:
    return w.problem["n_head"] * w.problem["n_speed"]


def action_tables(w):
    lib = load()
    na = n_actions(w)
    hx = np.zeros(na, np.float32)
    hy = np.zeros(na, np.float32)
    sp = np.zeros(na, np.float64)
    b = _Bound(w)
    lib.ora_action_tables(C.byref(b.p), _ptr(hx), _ptr(hy), _ptr(sp))
    return hx, hy, sp


def landing(w, t, c, r, a):
    lib = load()
    b = _Bound(w)
    ip, jp, ne = C.c_int32(), C.c_int32(), C.c_int32()
    lib.ora_landing(C.byref(b.p), C.byref(b.e), t, c, r, a, C.byref(ip), C.byref(jp), C.byref(ne))
    return ip.value, jp.value, bool(ne.value)


def row(w, t, c, a):
    """One (t, c, a) row: (cols, cnts, R[3], A[3], n_escape, n_near_edge)."""
    lib = load()
    b = _Bound(w)
    nr = w.problem["n_real"]
    cols = np.zeros(nr, np.int32)
    cnts = np.zeros(nr, np.int32)
    R = np.zeros(3)
    A = np.zeros(3)
    ne, nn = C.c_int64(0), C.c_int64(0)
    n = lib.ora_row(C.byref(b.p), C.byref(b.e), t, c, a, _ptr(cols), _ptr(cnts), _ptr(R), _ptr(A),
                    C.byref(ne), C.byref(nn))
    return cols[:n].copy(), cnts[:n].copy(), R, A, ne.value, nn.value


def build_model(w, cap: int | None = None) -> dict:
    """Full-domain model: CSR with counts, R and A as [3][rows], per-row near-edge counts."""
    lib = load()
    b = _Bound(w)
    rows = w.n_rows
    if cap is None:
        cap = max(rows * 4, 1024)
    while True:
        row_ptr = np.zeros(rows + 1, np.int64)
        col = np.zeros(cap, np.int32)
        cnt = np.zeros(cap, np.int32)
        R = np.zeros((3, rows))
        A = np.zeros((3, rows))
        row_near = np.zeros(rows, np.int32)
        ne, nn = C.c_int64(0), C.c_int64(0)
        nnz = lib.ora_build(C.byref(b.p), C.byref(b.e), _ptr(row_ptr), _ptr(col), _ptr(cnt), cap,
                            _ptr(R), _ptr(A), _ptr(row_near), C.byref(ne), C.byref(nn))
        if nnz <= cap:
            break
        cap = int(nnz)
    return dict(row_ptr=row_ptr, col=col[:nnz].copy(), cnt=cnt[:nnz].copy(), R=R, A=A,
                row_near=row_near, n_escape=ne.value, n_near_edge=nn.value, nnz=int(nnz))


def build_layers(w, t0: int, t1: int) -> dict:
    """The rows of the decision layers [t0, t1) only (row_ptr local to them, R and A
    [3][rows of the range]); concatenating the ranges in order gives build_model."""
    lib = load()
    b = _Bound(w)
    rows = (t1 - t0) * w.problem["nx"] * w.problem["ny"] * n_actions(w)
    cap = max(rows * 4, 1024)
    while True:
        row_ptr = np.zeros(rows + 1, np.int64)
        col = np.zeros(cap, np.int32)
        cnt = np.zeros(cap, np.int32)
        R = np.zeros((3, rows))
        A = np.zeros((3, rows))
        ne, nn = C.c_int64(0), C.c_int64(0)
        nnz = lib.ora_build_layers(C.byref(b.p), C.byref(b.e), t0, t1, _ptr(row_ptr), _ptr(col), _ptr(cnt), cap,
                                   _ptr(R), _ptr(A), None, C.byref(ne), C.byref(nn))
        if nnz <= cap:
            break
        cap = int(nnz)
    return dict(row_ptr=row_ptr, col=col[:nnz].copy(), cnt=cnt[:nnz].copy(), R=R, A=A, n_escape=ne.value,
                nnz=int(nnz))


def concat_layers(parts: list) -> dict:
    """One model from build_layers parts of consecutive layer ranges."""
    offs = np.cumsum([0] + [p["nnz"] for p in parts])
    row_ptr = np.concatenate([parts[0]["row_ptr"][:1]] + [p["row_ptr"][1:] + o for p, o in zip(parts, offs[:-1])])
    return dict(row_ptr=row_ptr, col=np.concatenate([p["col"] for p in parts]),
                cnt=np.concatenate([p["cnt"] for p in parts]), R=np.concatenate([p["R"] for p in parts], axis=1),
                A=np.concatenate([p["A"] for p in parts], axis=1), n_escape=sum(p["n_escape"] for p in parts),
                nnz=int(offs[-1]))


def backward(w, model: dict, mission: int):
    """Backward induction: (v, pi, w_abs) with w_abs the value of |rewards| under pi."""
    lib = load()
    p = problem_struct(w.problem)
    ns = w.n_states
    v = np.zeros(ns)
    pi = np.zeros(ns, np.int32)
    wa = np.zeros(ns)
    R = np.ascontiguousarray(model["R"][mission])
    A = np.ascontiguousarray(model["A"][mission])
    lib.ora_backward(C.byref(p), _ptr(model["row_ptr"]), _ptr(model["col"]), _ptr(model["cnt"]),
                     _ptr(R), _ptr(A), _ptr(v), _ptr(pi), _ptr(wa))
    return v, pi, wa


def jacobi(w, model: dict, mission: int, tol: float = 1e-6, max_sweeps: int = 100000, v0=None):
    lib = load()
    p = problem_struct(w.problem)
    v = np.zeros(w.n_states) if v0 is None else np.array(v0, np.float64)
    res = np.zeros(max_sweeps)
    R = np.ascontiguousarray(model["R"][mission])
    k = lib.ora_jacobi(C.byref(p), _ptr(model["row_ptr"]), _ptr(model["col"]), _ptr(model["cnt"]),
                       _ptr(R), tol, max_sweeps, _ptr(v), _ptr(res))
    return v, int(k), res[:k].copy()


def q_values(w, model: dict, mission: int, v, s_idx):
    lib = load()
    p = problem_struct(w.problem)
    s_idx = np.ascontiguousarray(s_idx, np.int64)
    q = np.zeros((len(s_idx), n_actions(w)))
    R = np.ascontiguousarray(model["R"][mission])
    v = np.ascontiguousarray(v, np.float64)
    lib.ora_q(C.byref(p), _ptr(model["row_ptr"]), _ptr(model["col"]), _ptr(model["cnt"]),
              _ptr(R), _ptr(v), _ptr(s_idx), len(s_idx), _ptr(q))
    return q


def max_speed(w):
    lib = load()
    b = _Bound(w)
    u, v = C.c_double(), C.c_double()
    lib.ora_max_speed(C.byref(b.p), C.byref(b.e), C.byref(u), C.byref(v))
    return u.value, v.value


def subgrid_auto(w):
    lib = load()
    b = _Bound(w)
    hx, hy = C.c_int32(), C.c_int32()
    lib.ora_subgrid_auto(C.byref(b.p), C.byref(b.e), C.byref(hx), C.byref(hy))
    return hx.value, hy.value


ROLL_ARRIVED, ROLL_OUTBOUND, ROLL_OBSTACLE, ROLL_HORIZON = 0, 1, 2, 3


def rollout(w, pi) -> dict:
    """Policy pi [n_states] followed from the start in every realization: per
    realization trajectory [n_real][nt+1], outcome, steps, returns [n_real][3],
    energy expended and speed sum; plus the ensemble statistics."""
    lib = load()
    b = _Bound(w)
    p = w.problem
    nr, nt = p["n_real"], p["nt"]
    pi = np.ascontiguousarray(pi, np.int32)
    traj = np.zeros((nr, nt + 1), np.int32)
    outcome = np.zeros(nr, np.int32)
    steps = np.zeros(nr, np.int32)
    ret = np.zeros((nr, 3))
    energy = np.zeros(nr)
    fsum = np.zeros(nr)
    lib.ora_rollout(C.byref(b.p), C.byref(b.e), _ptr(pi), _ptr(traj), _ptr(outcome), _ptr(steps), _ptr(ret),
                    _ptr(energy), _ptr(fsum))
    return dict(traj=traj, outcome=outcome, steps=steps, ret=ret, energy=energy, fsum=fsum,
                **rollout_summary(w, outcome, steps, ret, energy, fsum))


def rollout_summary(w, outcome, steps, ret, energy, fsum) -> dict:
    """Ensemble statistics of rollouts: P(reach), and over the arrived paths the
    mean travel time, energy expended, net energy consumed (energy expended
    minus energy harvested) and speed; the mean return of each mission over all
    paths. Plain sums in realization order."""
    p = w.problem
    arr = outcome == ROLL_ARRIVED
    n_arr = int(arr.sum())
    out = dict(n_real=len(outcome), n_arrived=n_arr, n_outbound=int((outcome == ROLL_OUTBOUND).sum()),
               n_obstacle=int((outcome == ROLL_OBSTACLE).sum()), n_horizon=int((outcome == ROLL_HORIZON).sum()),
               p_reach=n_arr / len(outcome))
    if n_arr:
        sa = steps[arr].astype(np.float64)
        out["mean_time_arrived"] = float(sum(sa) * p["dt"] / n_arr)
        out["mean_energy_arrived"] = float(sum(energy[arr]) / n_arr)
        # an arrived path's net-energy return is r_term minus its net consumption
        out["mean_net_energy_arrived"] = float(sum(p["r_term"] - ret[arr, 2]) / n_arr)
        out["mean_speed_arrived"] = float(sum(fsum[arr]) / sum(sa)) if sa.sum() > 0 else 0.0
    else:
        out.update(mean_time_arrived=0.0, mean_energy_arrived=0.0, mean_net_energy_arrived=0.0,
                   mean_speed_arrived=0.0)
    out["mean_return"] = [float(sum(ret[:, m]) / len(outcome)) for m in range(3)]
    return out


FLAG_SWEPT_PATH = 2


def segment_meets_cell(x0, y0, x1, y1, a, b) -> bool:
    return bool(load().ora_segment_meets_cell(x0, y0, x1, y1, a, b))
