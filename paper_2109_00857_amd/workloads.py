"""Seeded synthetic stochastic-flow planning workloads.

This module only produces input arrays: a reduced-order flow (mean, modes and
coefficients, Sec. II-C), a mean scalar field, an obstacle mask and the problem
parameters of Alg. 1's REQUIRE line (prob_type, prob_params, grid_params). It
contains none of the planner's arithmetic; the planner library and the CPU
oracle both consume the same arrays.

The paper's double-gyre forecast, radiation field and obstacle track (Sec. IV)
are not available, so these generators stand in for them. Shapes follow the
paper's application: a square basin, a 200x200x200 grid at the large end,
thousands of realizations, 16-32 headings.

Layouts (all C-contiguous):
  ubar, vbar : float32 [Tm][ny][nx]      Tm = nt if mean_time_varying else 1
  phiu, phiv : float32 [Tp][K][ny][nx]   Tp = nt if mode_time_varying else 1
  mu         : float32 [nt][K][n_real]   realization index fastest
  gbar       : float32 [nt+1][ny][nx]    or None when no net-energy mission
  mask       : uint8   [nt+1][ny][nx]    or None when there are no obstacles
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

MISSION_TIME = 0
MISSION_ENERGY = 1
MISSION_NET_ENERGY = 2
MISSION_NAMES = {MISSION_TIME: "time", MISSION_ENERGY: "energy", MISSION_NET_ENERGY: "net_energy"}

# RNG stream ids (Philox key word 1)
_S_MODES, _S_MU, _S_OBST, _S_MIX = 1, 2, 3, 4

# Reward constants (not given numerically in the paper; see Table I)
R_TERM = 100.0
R_OUTBOUND = -1000.0
C_F = 1.0
C_R = 1.0


def default_problem(**kw) -> dict:
    """A problem dict with every field the planner and the oracle read."""
    p = dict(
        nx=0, ny=0, nt=0, n_modes=0, n_real=0, n_head=0, n_speed=1,
        sub_hx=0, sub_hy=0, start_i=0, start_j=0, target_i=0, target_j=0,
        mean_time_varying=0, mode_time_varying=0,
        mission_mask=1 << MISSION_TIME, flags=0,
        dx=1.0, dy=1.0, dt=1.0, f_max=1.0,
        r_term=R_TERM, r_outbound=R_OUTBOUND, c_f=C_F, c_r=C_R,
    )
    p.update(kw)
    return p


@dataclass
class Workload:
    name: str
    problem: dict
    ubar: np.ndarray
    vbar: np.ndarray
    phiu: np.ndarray
    phiv: np.ndarray
    mu: np.ndarray
    gbar: np.ndarray | None = None
    mask: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n_actions(self) -> int:
        return self.problem["n_head"] * self.problem["n_speed"]

    @property
    def n_states(self) -> int:
        p = self.problem
        return p["nt"] * p["nx"] * p["ny"]

    @property
    def n_rows(self) -> int:
        return self.n_states * self.n_actions

    @property
    def nominal_samples(self) -> int:
        return self.n_rows * self.problem["n_real"]

    def missions(self) -> list[int]:
        m = self.problem["mission_mask"]
        return [k for k in range(3) if m >> k & 1]

    def check(self) -> None:
        p = self.problem
        nx, ny, nt, K, nr = p["nx"], p["ny"], p["nt"], p["n_modes"], p["n_real"]
        tm = nt if p["mean_time_varying"] else 1
        tp = nt if p["mode_time_varying"] else 1
        assert self.ubar.shape == (tm, ny, nx) and self.vbar.shape == (tm, ny, nx)
        assert self.phiu.shape == (tp, K, ny, nx) and self.phiv.shape == (tp, K, ny, nx)
        assert self.mu.shape == (nt, K, nr)
        for a in (self.ubar, self.vbar, self.phiu, self.phiv, self.mu):
            assert a.dtype == np.float32 and a.flags.c_contiguous
        if self.gbar is not None:
            assert self.gbar.shape == (nt + 1, ny, nx) and self.gbar.dtype == np.float32
        if p["mission_mask"] >> MISSION_NET_ENERGY & 1:
            assert self.gbar is not None
        if self.mask is not None:
            assert self.mask.shape == (nt + 1, ny, nx) and self.mask.dtype == np.uint8


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[seed, stream]))


def _centres(nx: int, ny: int):
    dx, dy = 1.0 / nx, 1.0 / ny
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    return np.meshgrid(x, y, indexing="xy")  # [ny][nx]


def _jet(nx: int, ny: int, width: float = 0.1, amp: float = 0.5):
    X, Y = _centres(nx, ny)
    u = amp * np.exp(-(((Y - 0.5) / width) ** 2))
    return u[None].astype(np.float32), np.zeros((1, ny, nx), np.float32)


def _normalise(pu: np.ndarray, pv: np.ndarray, dx: float, dy: float):
    """Scale each mode so that sum_c (phiu^2 + phiv^2) dx dy = 1 (fp64)."""
    n = np.sqrt(((pu ** 2 + pv ** 2).sum(axis=(-2, -1)) * dx * dy))
    return pu / n[..., None, None], pv / n[..., None, None]


def _sine_modes(nx: int, ny: int, K: int):
    """phi_k = sin(k pi x) sin(pi y); odd k (1-based) in u only, even k in v only."""
    X, Y = _centres(nx, ny)
    pu = np.zeros((K, ny, nx))
    pv = np.zeros((K, ny, nx))
    for k in range(1, K + 1):
        f = np.sin(k * np.pi * X) * np.sin(np.pi * Y)
        (pu if k % 2 == 1 else pv)[k - 1] = f
    pu, pv = _normalise(pu, pv, 1.0 / nx, 1.0 / ny)
    return pu[None].astype(np.float32), pv[None].astype(np.float32)


def _trig_modes(nx: int, ny: int, K: int, rng: np.random.Generator):
    """Each component of mode k is sin(a x + b) cos(c y + d), a, c ~ U[pi, 4pi], b, d ~ U[0, 2pi)."""
    X, Y = _centres(nx, ny)
    pu = np.zeros((K, ny, nx))
    pv = np.zeros((K, ny, nx))
    for k in range(K):
        for arr in (pu, pv):
            a, c = rng.uniform(np.pi, 4 * np.pi, size=2)
            b, d = rng.uniform(0.0, 2 * np.pi, size=2)
            arr[k] = np.sin(a * X + b) * np.cos(c * Y + d)
    pu, pv = _normalise(pu, pv, 1.0 / nx, 1.0 / ny)
    return pu[None].astype(np.float32), pv[None].astype(np.float32)


def _coeffs_iid(nt: int, K: int, nr: int, rng: np.random.Generator, s0: float = 0.2):
    sig = s0 / np.arange(1, K + 1)
    z = rng.standard_normal((nt, K, nr))
    return (z * sig[None, :, None]).astype(np.float32)


def _coeffs_ar1(nt: int, K: int, nr: int, rng: np.random.Generator, rho: float = 0.9, s0: float = 0.2):
    """Stationary AR(1) in t per (k, r): mu(0) = s xi, mu(t+1) = rho mu(t) + sqrt(1-rho^2) s xi."""
    sig = (s0 / np.arange(1, K + 1))[:, None]
    out = np.empty((nt, K, nr), np.float32)
    cur = sig * rng.standard_normal((K, nr))
    out[0] = cur
    q = math.sqrt(1.0 - rho * rho)
    for t in range(1, nt):
        cur = rho * cur + q * sig * rng.standard_normal((K, nr))
        out[t] = cur
    return out


def _gaussian_bump(nx: int, ny: int, nt: int):
    X, Y = _centres(nx, ny)
    g = np.empty((nt + 1, ny, nx), np.float32)
    for t in range(nt + 1):
        xb = 0.2 + 0.6 * t / nt
        g[t] = np.exp(-((X - xb) ** 2 + (Y - 0.5) ** 2) / (2 * 0.15 ** 2))
    return g


def _discs(nx, ny, nt, dt, start, target, rng, n=4):
    """Moving discs: radius U[.04,.08], centre U[.2,.8]^2, velocity U[-.2,.2]^2 per time unit."""
    X, Y = _centres(nx, ny)
    mask = np.zeros((nt + 1, ny, nx), np.uint8)
    tt = np.arange(nt + 1) * dt
    for _ in range(n):
        while True:
            rad = rng.uniform(0.04, 0.08)
            c0 = rng.uniform(0.2, 0.8, size=2)
            vel = rng.uniform(-0.2, 0.2, size=2)
            cx = c0[0] + vel[0] * tt
            cy = c0[1] + vel[1] * tt
            m = ((X[None] - cx[:, None, None]) ** 2 + (Y[None] - cy[:, None, None]) ** 2) <= rad * rad
            if not (m[:, start[1], start[0]].any() or m[:, target[1], target[0]].any()):
                break
        mask |= m.astype(np.uint8)
    return mask


def _blocks(nx, ny, nt, start, target, rng, n):
    """0-3 static square blocks of side U{1..ceil(n/8)}, clear of start and target."""
    mask = np.zeros((ny, nx), np.uint8)
    side_max = max(1, math.ceil(nx / 8))
    for _ in range(n):
        while True:
            s = int(rng.integers(1, side_max + 1))
            i0 = int(rng.integers(0, nx - s + 1))
            j0 = int(rng.integers(0, ny - s + 1))
            inside = lambda p: i0 <= p[0] < i0 + s and j0 <= p[1] < j0 + s
            if not (inside(start) or inside(target)):
                break
        mask[j0:j0 + s, i0:i0 + s] = 1
    return np.repeat(mask[None], nt + 1, axis=0)


def speed_bound(ubar, vbar, phiu, phiv, mu) -> float:
    """Upper bound on any synthesised component speed: per t, max over cells of
    |mean| + sum_k max_r |mu_k| |phi_k|, maximised over t and both components."""
    nt, K, _ = mu.shape
    m = np.abs(mu.astype(np.float64)).max(axis=2)  # [nt][K]
    best = 0.0
    for comp_mean, comp_mode in ((ubar, phiu), (vbar, phiv)):
        am = np.abs(comp_mean.astype(np.float64))
        ap = np.abs(comp_mode.astype(np.float64))
        for t in range(nt):
            mt = am[t if am.shape[0] > 1 else 0]
            pt = ap[t if ap.shape[0] > 1 else 0]
            s = mt + np.tensordot(m[t], pt, axes=(0, 0))
            best = max(best, float(s.max()))
    return best


def config1(seed: int = 0, nx: int = 25, ny: int = 25, nt: int = 20, n_real: int = 500,
            n_head: int = 8, sub_h: int | None = None) -> Workload:
    """Small plain case: 25x25, T=20, dt=0.05, jet + 4 sine modes, 500 iid realizations,
    8 headings at F=0.3, a static 3x3 block, time mission, corner to corner."""
    ubar, vbar = _jet(nx, ny)
    phiu, phiv = _sine_modes(nx, ny, 4)
    mu = _coeffs_iid(nt, 4, n_real, _rng(seed, _S_MU))
    mask = np.zeros((nt + 1, ny, nx), np.uint8)
    lo, hi = (11 * nx) // 25, (13 * nx) // 25
    mask[:, lo:hi + 1, lo:hi + 1] = 1
    p = default_problem(nx=nx, ny=ny, nt=nt, n_modes=4, n_real=n_real, n_head=n_head, n_speed=1,
                        start_i=0, start_j=0, target_i=nx - 1, target_j=ny - 1,
                        mission_mask=1 << MISSION_TIME, dx=1.0 / nx, dy=1.0 / ny, dt=0.05, f_max=0.3)
    if sub_h is not None:
        p["sub_hx"] = p["sub_hy"] = sub_h
    w = Workload("c1_small", p, ubar, vbar, phiu, phiv, mu, None, mask,
                 meta=dict(seed=seed, sub_grid="auto" if sub_h is None else sub_h))
    w.check()
    return w


def _paper_shaped(name, seed, nx, ny, nt, K, n_real, n_head, h, missions, rho=0.9):
    rng_modes = _rng(seed, _S_MODES)
    ubar, vbar = _jet(nx, ny)
    phiu, phiv = _trig_modes(nx, ny, K, rng_modes)
    mu = _coeffs_ar1(nt, K, n_real, _rng(seed, _S_MU), rho=rho)
    f_max = 0.3
    M = speed_bound(ubar, vbar, phiu, phiv, mu)
    lam = (h + 0.5) * (1.0 - 1e-3) / (M + f_max)
    dx, dy = 1.0 / nx, 1.0 / ny
    dt = lam * dx
    start = (nx // 2, int(0.2 * ny))
    target = (nx // 2, int(0.8 * ny))
    mask = _discs(nx, ny, nt, dt, start, target, _rng(seed, _S_OBST))
    mm = 0
    for m in missions:
        mm |= 1 << m
    gbar = _gaussian_bump(nx, ny, nt) if (mm >> MISSION_NET_ENERGY & 1) else None
    p = default_problem(nx=nx, ny=ny, nt=nt, n_modes=K, n_real=n_real, n_head=n_head, n_speed=1,
                        sub_hx=h, sub_hy=h, start_i=start[0], start_j=start[1],
                        target_i=target[0], target_j=target[1], mission_mask=mm,
                        dx=dx, dy=dy, dt=dt, f_max=f_max)
    w = Workload(name, p, ubar, vbar, phiu, phiv, mu, gbar, mask,
                 meta=dict(seed=seed, speed_bound=M, lam=lam))
    w.check()
    return w


def config2(seed: int = 0, nx: int = 100, ny: int = 100, nt: int = 120, n_real: int = 5000,
            K: int = 10, n_head: int = 16, missions=(0, 1, 2)) -> Workload:
    """Paper-shaped single instance: 100x100, T=120, 10 trig modes, 5000 AR(1) realizations,
    16 headings, 5x5 sub-grid, 4 moving discs, all three missions."""
    return _paper_shaped("c2_paper_shaped", seed, nx, ny, nt, K, n_real, n_head, 2, missions)


def config3(seed: int = 0, nx: int = 200, ny: int = 200, nt: int = 200, n_real: int = 10000,
            K: int = 16, n_head: int = 32, missions=(2,)) -> Workload:
    """Large single instance: 200x200, T=200, 16 modes, 10000 realizations, 32 headings,
    7x7 sub-grid, net-energy mission."""
    return _paper_shaped("c3_large", seed, nx, ny, nt, K, n_real, n_head, 3, missions)


def batched_instance(i: int, base_seed: int = 1000) -> Workload:
    """One of the uneven batched instances: n ~ U{20..120}, T ~ U{20..120}, K ~ U{4..12},
    N_r ~ U{500..5000}, headings ~ U{8..16}, jet width ~ U[.05,.2], 0-3 static blocks,
    corner to corner, random mission, lambda = 1.25, sub-grid from a speed bound."""
    seed = base_seed + i
    r = _rng(seed, _S_MIX)
    n = int(r.integers(20, 121))
    nt = int(r.integers(20, 121))
    K = int(r.integers(4, 13))
    nr = int(r.integers(500, 5001))
    nh = int(r.integers(8, 17))
    width = float(r.uniform(0.05, 0.2))
    mission = int(r.integers(0, 3))
    nblk = int(r.integers(0, 4))
    ubar, vbar = _jet(n, n, width=width)
    phiu, phiv = _sine_modes(n, n, K)
    mu = _coeffs_iid(nt, K, nr, _rng(seed, _S_MU))
    start, target = (0, 0), (n - 1, n - 1)
    mask = _blocks(n, n, nt, start, target, _rng(seed, _S_OBST), nblk) if nblk else None
    dx = 1.0 / n
    dt = 1.25 * dx
    gbar = _gaussian_bump(n, n, nt) if mission == MISSION_NET_ENERGY else None
    p = default_problem(nx=n, ny=n, nt=nt, n_modes=K, n_real=nr, n_head=nh, n_speed=1,
                        start_i=0, start_j=0, target_i=n - 1, target_j=n - 1,
                        mission_mask=1 << mission, dx=dx, dy=dx, dt=dt, f_max=0.3)
    w = Workload(f"batched_{i}", p, ubar, vbar, phiu, phiv, mu, gbar, mask,
                 meta=dict(seed=seed, jet_width=width))
    w.check()
    return w


def uniform_flow(nx: int, ny: int, nt: int, u0: float, v0: float, n_real: int, n_head: int,
                 f_max: float, dx: float = 1.0, dy: float = 1.0, dt: float = 1.0,
                 sigma: float = 0.0, mode_u: float = 1.0, mode_v: float = 0.0, seed: int = 0,
                 start=(0, 0), target=(1, 1), sub_h: int = 2, mission_mask: int = 1,
                 mask: np.ndarray | None = None, gbar: np.ndarray | None = None,
                 n_speed: int = 1) -> Workload:
    """Spatially uniform mean flow (u0, v0) plus one constant mode (mode_u, mode_v) whose
    coefficient is N(0, sigma^2) per (t, r); sigma = 0 gives a deterministic flow.
    The mode is passed as given (not normalised)."""
    ubar = np.full((1, ny, nx), u0, np.float32)
    vbar = np.full((1, ny, nx), v0, np.float32)
    phiu = np.full((1, 1, ny, nx), mode_u, np.float32)
    phiv = np.full((1, 1, ny, nx), mode_v, np.float32)
    if sigma > 0:
        mu = (sigma * _rng(seed, _S_MU).standard_normal((nt, 1, n_real))).astype(np.float32)
    else:
        mu = np.zeros((nt, 1, n_real), np.float32)
    p = default_problem(nx=nx, ny=ny, nt=nt, n_modes=1, n_real=n_real, n_head=n_head, n_speed=n_speed,
                        sub_hx=sub_h, sub_hy=sub_h, start_i=start[0], start_j=start[1],
                        target_i=target[0], target_j=target[1], mission_mask=mission_mask,
                        dx=dx, dy=dy, dt=dt, f_max=f_max)
    w = Workload("uniform_flow", p, ubar, vbar, phiu, phiv, mu, gbar, mask)
    w.check()
    return w


CONFIGS = {"c1": config1, "c2": config2, "c3": config3}
