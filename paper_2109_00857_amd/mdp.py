"""Python binding of libmdp.so (include/mdp.h): argument marshalling only.

Every computation runs in the HIP kernels behind the C ABI. PyTorch supplies
device memory and streams. The functions named like the C entry points
(``mdp_build``, ``mdp_value_iterate``, ``mdp_policy``, ...) pass their
arguments straight through; ``Planner`` adds allocation conveniences on top.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmdp.so")

MDP_OK = 0
MDP_E_INVALID = 1
MDP_E_CAPACITY = 2
MDP_E_SUBGRID = 3
MDP_E_HIP = 4
MDP_E_NOT_CONVERGED = 5
MDP_E_SCRATCH = 6
MDP_FLAG_NEAR_EDGE = 1
MDP_FLAG_SWEPT_PATH = 2
MISSION_TIME, MISSION_ENERGY, MISSION_NET_ENERGY = 0, 1, 2


class MdpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class MdpProblem(C.Structure):
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


class MdpEnv(C.Structure):
    _fields_ = [("ubar", C.c_void_p), ("vbar", C.c_void_p), ("phiu", C.c_void_p),
                ("phiv", C.c_void_p), ("mu", C.c_void_p), ("gbar", C.c_void_p), ("mask", C.c_void_p)]


class MdpModel(C.Structure):
    _fields_ = [("row_ptr", C.c_void_p), ("col", C.c_void_p), ("cnt", C.c_void_p),
                ("reward", C.c_void_p), ("nnz_capacity", C.c_int64), ("ent", C.c_void_p),
                ("roff", C.c_void_p)]


class MdpSizes(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("n_states", "n_actions", "n_rows", "n_sg", "nnz_upper",
                                          "n_missions", "scratch_bytes", "env_bytes", "layers_per_slab")]


class MdpBuildStats(C.Structure):
    _fields_ = [("samples", C.c_int64), ("nnz", C.c_int64), ("n_escape", C.c_int64),
                ("n_near_edge", C.c_int64), ("status", C.c_int32), ("n_slabs", C.c_int32)]


class MdpViStats(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("status", C.c_int32), ("residual", C.c_double)]


_lib = None


MDP_MAX_TUNE = 18


class MdpTuneReport(C.Structure):
    _fields_ = [("n_candidates", C.c_int32), ("best", C.c_int32), ("sample_layers", C.c_int32),
                ("default_shape", C.c_int32), ("row_lanes", C.c_int32 * MDP_MAX_TUNE), ("rch", C.c_int32 * MDP_MAX_TUNE),
                ("pack16", C.c_int32 * MDP_MAX_TUNE), ("ms", C.c_double * MDP_MAX_TUNE)]


MDP_ROLL_ARRIVED, MDP_ROLL_OUTBOUND, MDP_ROLL_OBSTACLE, MDP_ROLL_HORIZON = 0, 1, 2, 3


class MdpRolloutPath(C.Structure):
    _fields_ = [("outcome", C.c_int32), ("steps", C.c_int32), ("ret", C.c_double * 3), ("energy", C.c_double),
                ("fsum", C.c_double)]


class MdpRolloutStats(C.Structure):
    _fields_ = [("n_real", C.c_int64), ("n_arrived", C.c_int64), ("n_outbound", C.c_int64),
                ("n_obstacle", C.c_int64), ("n_horizon", C.c_int64), ("p_reach", C.c_double),
                ("mean_time_arrived", C.c_double), ("mean_energy_arrived", C.c_double),
                ("mean_net_energy_arrived", C.c_double), ("mean_speed_arrived", C.c_double),
                ("mean_return", C.c_double * 3)]


class MdpServerConfig(C.Structure):
    _fields_ = [("max_inflight", C.c_int32), ("sweeps_per_step", C.c_int32), ("max_sweeps", C.c_int32),
                ("build_share", C.c_int32), ("tol", C.c_double), ("chunk_cost", C.c_double),
                ("large_cost", C.c_double)]


class MdpServed(C.Structure):
    _fields_ = [("tag", C.c_int64), ("nnz", C.c_int64), ("samples", C.c_int64), ("admit_step", C.c_int64),
                ("done_step", C.c_int64), ("residual", C.c_double), ("v_start", C.c_double),
                ("status", C.c_int32), ("build_status", C.c_int32), ("sweeps", C.c_int32), ("pad", C.c_int32)]


class MdpServerState(C.Structure):
    _fields_ = [("queued", C.c_int32), ("in_flight", C.c_int32), ("completed", C.c_int32), ("pad", C.c_int32),
                ("pool_used", C.c_int64), ("steps", C.c_int64)]


def load():
    """Load libmdp.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        lib = C.CDLL(LIB_PATH)
        vp, P = C.c_void_p, C.POINTER(MdpProblem)
        sigs = {
            "mdp_ctx_create": ([C.c_int32, C.POINTER(vp)], C.c_int32),
            "mdp_ctx_destroy": ([vp], C.c_int32),
            "mdp_status_str": ([C.c_int32], C.c_char_p),
            "mdp_last_error": ([vp], C.c_char_p),
            "mdp_build_query": ([P, C.POINTER(MdpSizes)], C.c_int32),
            "mdp_subgrid_auto": ([vp, P, C.POINTER(MdpEnv), C.POINTER(C.c_int32), C.POINTER(C.c_int32), vp],
                                 C.c_int32),
            "mdp_build": ([vp, P, C.POINTER(MdpEnv), C.POINTER(MdpModel), vp, C.c_size_t, vp, vp], C.c_int32),
            "mdp_build_sync": ([vp, vp, vp], C.c_int32),
            "mdp_build_from": ([vp, P, C.POINTER(MdpEnv), C.POINTER(MdpModel), C.c_int32, vp, C.c_size_t, vp, vp],
                               C.c_int32),
            "mdp_value_iterate_layers": ([vp, P, C.POINTER(MdpModel), C.c_int32, C.c_int32, C.c_double, C.c_int32, vp,
                                          vp, C.c_size_t, vp, vp], C.c_int32),
            "mdp_value_iterate": ([vp, P, C.POINTER(MdpModel), C.c_int32, C.c_double, C.c_int32, vp, vp,
                                   C.c_size_t, vp, vp], C.c_int32),
            "mdp_value_iterate_noalloc": ([vp, P, C.POINTER(MdpModel), C.c_int32, C.c_double, C.c_int32, vp, vp, vp],
                                          C.c_int32),
            "mdp_value_iterate_missions": ([vp, P, C.POINTER(MdpModel), C.c_int32, C.POINTER(C.c_int32),
                                            C.c_double, C.c_int32, C.POINTER(vp), vp, C.c_size_t, vp, vp],
                                           C.c_int32),
            "mdp_policy": ([vp, P, C.POINTER(MdpModel), C.c_int32, vp, vp, vp], C.c_int32),
            "mdp_rollout_query": ([P, C.POINTER(C.c_size_t)], C.c_int32),
            "mdp_rollout": ([vp, P, C.POINTER(MdpEnv), vp, vp, vp, vp, C.c_size_t, vp, vp], C.c_int32),
            "mdp_batch_query": ([C.c_int32, P, C.c_int64, C.POINTER(C.c_size_t)], C.c_int32),
            "mdp_batch_create": ([vp, C.c_int32, P, C.POINTER(MdpEnv), C.POINTER(MdpModel), vp, vp, vp, C.c_int64,
                                  vp, C.c_size_t, C.POINTER(vp)], C.c_int32),
            "mdp_batch_build": ([vp, vp], C.c_int32),
            "mdp_batch_solve": ([vp, C.c_double, C.c_int32, vp], C.c_int32),
            "mdp_batch_stats": ([vp, vp, vp], C.c_int32),
            "mdp_batch_capture": ([vp, C.c_double, C.c_int32, vp], C.c_int32),
            "mdp_batch_replay": ([vp, vp], C.c_int32),
            "mdp_batch_destroy": ([vp], C.c_int32),
            "mdp_autotune_query": ([P, C.POINTER(C.c_size_t)], C.c_int32),
            "mdp_autotune": ([vp, P, C.POINTER(MdpEnv), vp, C.c_size_t, C.POINTER(MdpTuneReport), vp], C.c_int32),
            "mdp_ctx_set_plan": ([vp, P, C.c_int32, C.c_int32, C.c_int32], C.c_int32),
            "mdp_server_footprint": ([P, C.POINTER(C.c_size_t)], C.c_int32),
            "mdp_server_create": ([vp, C.POINTER(MdpServerConfig), vp, C.c_size_t, C.POINTER(vp)], C.c_int32),
            "mdp_server_submit": ([vp, P, C.POINTER(MdpEnv), C.c_int32, vp, vp, C.c_int64], C.c_int32),
            "mdp_server_step": ([vp, vp, C.POINTER(C.c_int32)], C.c_int32),
            "mdp_server_poll": ([vp, C.POINTER(MdpServed), C.c_int32, C.POINTER(C.c_int32)], C.c_int32),
            "mdp_server_info": ([vp, C.POINTER(MdpServerState)], C.c_int32),
            "mdp_server_destroy": ([vp], C.c_int32),
            "mdp_ctx_profile": ([vp, C.c_int32], C.c_int32),
            "mdp_ctx_profile_read": ([vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)], C.c_int32),
        }
        for name, (args, res) in sigs.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _lib = lib
    return _lib


EXPORTED = ["mdp_ctx_create", "mdp_ctx_destroy", "mdp_status_str", "mdp_last_error", "mdp_build_query",
            "mdp_subgrid_auto", "mdp_build", "mdp_build_sync", "mdp_build_from", "mdp_value_iterate",
            "mdp_value_iterate_layers", "mdp_value_iterate_noalloc", "mdp_value_iterate_missions",
            "mdp_policy", "mdp_rollout_query", "mdp_rollout",
            "mdp_ctx_profile",
            "mdp_ctx_profile_read", "mdp_batch_query", "mdp_batch_create", "mdp_batch_build", "mdp_batch_solve",
            "mdp_batch_stats", "mdp_batch_capture", "mdp_batch_replay", "mdp_batch_destroy",
            "mdp_server_footprint", "mdp_server_create", "mdp_server_submit", "mdp_server_step",
            "mdp_server_poll", "mdp_server_info", "mdp_server_destroy", "mdp_autotune_query", "mdp_autotune",
            "mdp_ctx_set_plan"]
MDP_KERNEL_BUILD, MDP_KERNEL_VI_SWEEP, MDP_KERNEL_POLICY, MDP_KERNEL_COPY = 0, 1, 2, 3


def problem_struct(p: dict) -> MdpProblem:
    return MdpProblem(**{k: p[k] for k, _ in MdpProblem._fields_})


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------- C entry points
def mdp_status_str(status: int) -> str:
    return load().mdp_status_str(status).decode()


def mdp_ctx_create(device: int = 0):
    h = C.c_void_p()
    rc = load().mdp_ctx_create(device, C.byref(h))
    if rc != MDP_OK:
        raise MdpError(rc, f"mdp_ctx_create: {mdp_status_str(rc)}")
    return h


def mdp_ctx_destroy(ctx) -> None:
    load().mdp_ctx_destroy(ctx)


def mdp_last_error(ctx) -> str:
    return load().mdp_last_error(ctx).decode()


def mdp_build_query(problem: dict) -> dict:
    s = MdpSizes()
    rc = load().mdp_build_query(C.byref(problem_struct(problem)), C.byref(s))
    if rc != MDP_OK:
        raise MdpError(rc, "mdp_build_query: invalid problem")
    return {k: getattr(s, k) for k, _ in MdpSizes._fields_}


def _check(ctx, rc, what):
    if rc != MDP_OK:
        raise MdpError(rc, f"{what}: {mdp_status_str(rc)}: {mdp_last_error(ctx)}")


def mdp_subgrid_auto(ctx, problem: dict, env: dict, stream=None):
    hx, hy = C.c_int32(), C.c_int32()
    e = MdpEnv(*[_ptr(env.get(k)) for k, _ in MdpEnv._fields_])
    rc = load().mdp_subgrid_auto(ctx, C.byref(problem_struct(problem)), C.byref(e), C.byref(hx),
                                 C.byref(hy), _stream_handle(stream))
    _check(ctx, rc, "mdp_subgrid_auto")
    return hx.value, hy.value


def mdp_build(ctx, problem: dict, env: dict, model: dict, scratch: torch.Tensor, stats: torch.Tensor,
              stream=None) -> None:
    """Enqueue the build; `stats` is a (pinned) uint8 host tensor of sizeof(mdp_build_stats)."""
    e = MdpEnv(*[_ptr(env.get(k)) for k, _ in MdpEnv._fields_])
    m = _model_struct(model)
    rc = load().mdp_build(ctx, C.byref(problem_struct(problem)), C.byref(e), C.byref(m), _ptr(scratch),
                          scratch.numel(), stats.data_ptr(), _stream_handle(stream))
    _check(ctx, rc, "mdp_build")


def mdp_build_from(ctx, problem: dict, env: dict, model: dict, t0: int, scratch: torch.Tensor, stats: torch.Tensor,
                   stream=None) -> None:
    """Enqueue the rebuild of layers [t0, nt) of a built model after the environment changed."""
    e = MdpEnv(*[_ptr(env.get(k)) for k, _ in MdpEnv._fields_])
    m = _model_struct(model)
    rc = load().mdp_build_from(ctx, C.byref(problem_struct(problem)), C.byref(e), C.byref(m), t0, _ptr(scratch),
                               scratch.numel(), stats.data_ptr(), _stream_handle(stream))
    _check(ctx, rc, "mdp_build_from")


def mdp_value_iterate_layers(ctx, problem: dict, model: dict, mission: int, t_first: int, tol: float,
                             max_sweeps: int, v: torch.Tensor, scratch: torch.Tensor, stats: torch.Tensor,
                             stream=None) -> None:
    m = _model_struct(model)
    rc = load().mdp_value_iterate_layers(ctx, C.byref(problem_struct(problem)), C.byref(m), mission, t_first, tol,
                                         max_sweeps, _ptr(v), _ptr(scratch), scratch.numel(), stats.data_ptr(),
                                         _stream_handle(stream))
    _check(ctx, rc, "mdp_value_iterate_layers")


def mdp_build_sync(ctx, stats: torch.Tensor, stream=None) -> int:
    """Wait for the build on `stream`; return its device status (MDP_OK, MDP_E_CAPACITY,
    MDP_E_SUBGRID) without raising for those two."""
    rc = load().mdp_build_sync(ctx, stats.data_ptr(), _stream_handle(stream))
    if rc not in (MDP_OK, MDP_E_CAPACITY, MDP_E_SUBGRID):
        _check(ctx, rc, "mdp_build_sync")
    return rc


def mdp_value_iterate(ctx, problem: dict, model: dict, mission: int, tol: float, max_sweeps: int,
                      v: torch.Tensor, scratch: torch.Tensor, stats: torch.Tensor, stream=None) -> None:
    m = _model_struct(model)
    rc = load().mdp_value_iterate(ctx, C.byref(problem_struct(problem)), C.byref(m), mission, tol, max_sweeps,
                                  _ptr(v), _ptr(scratch), scratch.numel(), stats.data_ptr(),
                                  _stream_handle(stream))
    _check(ctx, rc, "mdp_value_iterate")


def mdp_value_iterate_noalloc(ctx, problem: dict, model: dict, mission: int, tol: float, max_sweeps: int,
                              v: torch.Tensor, stats: torch.Tensor, stream=None) -> None:
    """mdp_value_iterate on the library's static per-GPU scratch (no allocation)."""
    m = _model_struct(model)
    rc = load().mdp_value_iterate_noalloc(ctx, C.byref(problem_struct(problem)), C.byref(m), mission, tol,
                                          max_sweeps, _ptr(v), stats.data_ptr(), _stream_handle(stream))
    _check(ctx, rc, "mdp_value_iterate_noalloc")


MDP_NOALLOC_SCRATCH_BYTES = 72 << 20


def mdp_value_iterate_missions(ctx, problem: dict, model: dict, missions, tol: float, max_sweeps: int,
                               vs, scratch: torch.Tensor, stats: torch.Tensor, stream=None) -> None:
    """Several missions of one model in one solve; ``stats`` holds len(missions) MdpViStats."""
    n = len(missions)
    m = _model_struct(model)
    ms = (C.c_int32 * n)(*missions)
    ptrs = (C.c_void_p * n)(*[_ptr(v) for v in vs])
    rc = load().mdp_value_iterate_missions(ctx, C.byref(problem_struct(problem)), C.byref(m), n, ms, tol,
                                           max_sweeps, ptrs, _ptr(scratch), scratch.numel(), stats.data_ptr(),
                                           _stream_handle(stream))
    _check(ctx, rc, "mdp_value_iterate_missions")


def mdp_policy(ctx, problem: dict, model: dict, mission: int, v: torch.Tensor, pi: torch.Tensor,
               stream=None) -> None:
    m = _model_struct(model)
    rc = load().mdp_policy(ctx, C.byref(problem_struct(problem)), C.byref(m), mission, _ptr(v), _ptr(pi),
                           _stream_handle(stream))
    _check(ctx, rc, "mdp_policy")


def mdp_rollout_query(problem: dict) -> int:
    n = C.c_size_t()
    rc = load().mdp_rollout_query(C.byref(problem_struct(problem)), C.byref(n))
    if rc != MDP_OK:
        raise MdpError(rc, "mdp_rollout_query: invalid problem")
    return n.value


def mdp_rollout(ctx, problem: dict, env: dict, pi: torch.Tensor, traj, paths, scratch: torch.Tensor,
                stats: torch.Tensor, stream=None) -> None:
    """Enqueue the rollout of policy `pi`; `stats` is a (pinned) uint8 host tensor of
    sizeof(mdp_rollout_stats); traj (int32 [nt+1][n_real]) and paths may be None."""
    e = MdpEnv(*[_ptr(env.get(k)) for k, _ in MdpEnv._fields_])
    rc = load().mdp_rollout(ctx, C.byref(problem_struct(problem)), C.byref(e), _ptr(pi), _ptr(traj), _ptr(paths),
                            _ptr(scratch), scratch.numel(), stats.data_ptr(), _stream_handle(stream))
    _check(ctx, rc, "mdp_rollout")


def rollout_stats_dict(buf: torch.Tensor) -> dict:
    s = MdpRolloutStats.from_buffer_copy(bytes(buf.numpy()))
    out = {k: getattr(s, k) for k, _ in MdpRolloutStats._fields_}
    out["mean_return"] = list(s.mean_return)
    return out


def mdp_ctx_profile(ctx, enable: bool) -> None:
    _check(ctx, load().mdp_ctx_profile(ctx, 1 if enable else 0), "mdp_ctx_profile")


def mdp_ctx_profile_read(ctx, kernel: int):
    n, ms = C.c_int64(), C.c_double()
    _check(ctx, load().mdp_ctx_profile_read(ctx, kernel, C.byref(n), C.byref(ms)), "mdp_ctx_profile_read")
    return n.value, ms.value


def stats_buffer(cls) -> torch.Tensor:
    return torch.zeros(C.sizeof(cls), dtype=torch.uint8, pin_memory=True)


def read_stats(buf: torch.Tensor, cls) -> dict:
    s = cls.from_buffer_copy(bytes(buf.numpy()))
    return {k: getattr(s, k) for k, _ in cls._fields_}


# ---------------------------------------------------------------- conveniences
class Planner:
    """A context on one device plus allocation helpers (all device memory from torch)."""

    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        self.ctx = mdp_ctx_create(device)

    def close(self):
        if self.ctx is not None:
            mdp_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def upload_env(self, w) -> dict:
        d = self.device
        env = {k: torch.from_numpy(np.ascontiguousarray(getattr(w, k))).to(d)
               for k in ("ubar", "vbar", "phiu", "phiv", "mu")}
        env["gbar"] = None if w.gbar is None else torch.from_numpy(w.gbar).to(d)
        env["mask"] = None if w.mask is None else torch.from_numpy(w.mask).to(d)
        return env

    def alloc_model(self, problem: dict, capacity: int, packed: bool = False) -> dict:
        """Model buffers for `capacity` nonzeros; with `packed`, also the fused sweep's
        packed entries and row offsets (mdp_build fills them)."""
        sz = mdp_build_query(problem)
        d = self.device
        m = dict(
            row_ptr=torch.empty(sz["n_rows"] + 1, dtype=torch.int64, device=d),
            col=torch.empty(max(capacity, 1), dtype=torch.int32, device=d),
            cnt=torch.empty(max(capacity, 1), dtype=torch.uint16, device=d),
            reward=torch.empty((sz["n_missions"], sz["n_rows"]), dtype=torch.float32, device=d),
        )
        if packed:
            m["ent"] = torch.empty(max(capacity, 1), dtype=torch.int32, device=d)
            m["roff"] = torch.empty(max(sz["n_rows"], 1), dtype=torch.uint16, device=d)
        return m

    def scratch(self, problem: dict) -> torch.Tensor:
        sz = mdp_build_query(problem)
        return torch.empty(sz["scratch_bytes"], dtype=torch.uint8, device=self.device)

    def build(self, problem: dict, env: dict, capacity: int | None = None, scratch=None, stream=None,
              packed: bool = True):
        """Build with a capacity guess; rebuild once with the exact nnz if it was too small.
        With `packed` the model also holds the fused sweep's packed entries.
        Returns (model, stats). Synchronises the stream."""
        sz = mdp_build_query(problem)
        if capacity is None:
            capacity = min(sz["nnz_upper"], 4 * sz["n_rows"] + 1024)
        if scratch is None:
            scratch = self.scratch(problem)
        for _ in range(2):
            model = self.alloc_model(problem, capacity, packed)
            st = stats_buffer(MdpBuildStats)
            mdp_build(self.ctx, problem, env, model, scratch, st, stream)
            mdp_build_sync(self.ctx, st, stream)
            stats = read_stats(st, MdpBuildStats)
            if stats["status"] != MDP_E_CAPACITY:
                break
            capacity = stats["nnz"]
        if stats["status"] == MDP_OK:
            for k in ("col", "cnt", "ent"):
                if k in model:
                    model[k] = model[k][: stats["nnz"]]
        return model, stats

    def value_iterate(self, problem: dict, model: dict, mission: int, tol: float = 1e-6,
                      max_sweeps: int = 100000, v0=None, scratch=None, stream=None):
        ns = mdp_build_query(problem)["n_states"]
        v = torch.zeros(ns, dtype=torch.float64, device=self.device) if v0 is None else v0.clone()
        if scratch is None:
            scratch = self.scratch(problem)
        st = stats_buffer(MdpViStats)
        mdp_value_iterate(self.ctx, problem, model, mission, tol, max_sweeps, v, scratch, st, stream)
        (stream or torch.cuda.current_stream()).synchronize()
        return v, read_stats(st, MdpViStats)

    def value_iterate_missions(self, problem: dict, model: dict, missions, tol: float = 1e-6,
                               max_sweeps: int = 100000, v0s=None, scratch=None, stream=None):
        """Returns ([v per mission], [stats per mission]); synchronises the stream."""
        ns = mdp_build_query(problem)["n_states"]
        n = len(missions)
        if v0s is None:
            vs = [torch.zeros(ns, dtype=torch.float64, device=self.device) for _ in range(n)]
        else:
            vs = [v.clone() for v in v0s]
        if scratch is None:
            scratch = torch.empty(n * mdp_build_query(problem)["scratch_bytes"], dtype=torch.uint8,
                                  device=self.device)
        st = torch.zeros(n * C.sizeof(MdpViStats), dtype=torch.uint8, pin_memory=True)
        mdp_value_iterate_missions(self.ctx, problem, model, missions, tol, max_sweeps, vs, scratch, st, stream)
        (stream or torch.cuda.current_stream()).synchronize()
        k = C.sizeof(MdpViStats)
        return vs, [read_stats(st[i * k:(i + 1) * k], MdpViStats) for i in range(n)]

    def policy(self, problem: dict, model: dict, mission: int, v: torch.Tensor, stream=None):
        ns = mdp_build_query(problem)["n_states"]
        pi = torch.empty(ns, dtype=torch.int32, device=self.device)
        mdp_policy(self.ctx, problem, model, mission, v, pi, stream)
        return pi

    def rollout(self, problem: dict, env: dict, pi: torch.Tensor, keep_traj: bool = True, stream=None):
        """Roll pi out in every realization. Returns (traj [nt+1][n_real] or None,
        paths as a dict of numpy arrays, stats dict); synchronises the stream."""
        nr, nt = problem["n_real"], problem["nt"]
        traj = torch.empty((nt + 1, nr), dtype=torch.int32, device=self.device) if keep_traj else None
        paths = torch.empty(nr * C.sizeof(MdpRolloutPath), dtype=torch.uint8, device=self.device)
        scratch = torch.empty(mdp_rollout_query(problem), dtype=torch.uint8, device=self.device)
        st = stats_buffer(MdpRolloutStats)
        mdp_rollout(self.ctx, problem, env, pi, traj, paths, scratch, st, stream)
        (stream or torch.cuda.current_stream()).synchronize()
        raw = np.frombuffer(paths.cpu().numpy().tobytes(), dtype=np.dtype(
            [("outcome", "<i4"), ("steps", "<i4"), ("ret", "<f8", (3,)), ("energy", "<f8"), ("fsum", "<f8")]))
        pd = {k: np.ascontiguousarray(raw[k]) for k in ("outcome", "steps", "ret", "energy", "fsum")}
        return traj, pd, rollout_stats_dict(st)


# ---------------------------------------------------------------- batches
def _model_struct(m: dict) -> MdpModel:
    """The C view of a model dict; "ent" and "roff" (the fused sweep's packed entries
    and 16-bit row offsets) are optional, together."""
    return MdpModel(_ptr(m["row_ptr"]), _ptr(m["col"]), _ptr(m["cnt"]), _ptr(m["reward"]), int(m["col"].numel()),
                    _ptr(m.get("ent")), _ptr(m.get("roff")))


def mdp_batch_query(problems: list, pool_entries: int = 0) -> int:
    arr = (MdpProblem * len(problems))(*[problem_struct(p) for p in problems])
    out = C.c_size_t()
    rc = load().mdp_batch_query(len(problems), arr, pool_entries, C.byref(out))
    if rc != MDP_OK:
        raise MdpError(rc, "mdp_batch_query: invalid batch")
    return out.value


class Batch:
    """Many problems built in one persistent launch and solved with one sweep
    launch per iteration (include/mdp.h, mdp_batch_*). Allocates models,
    values, policies and scratch with torch; recreates itself once if a model
    or the staging pool was too small."""

    def __init__(self, planner: "Planner", problems: list, envs: list, missions: list, pool_entries: int = 0,
                 capacities: list | None = None):
        self.pl, self.problems, self.envs, self.missions = planner, problems, envs, list(missions)
        self.n = len(problems)
        self.h = None
        sizes = [mdp_build_query(p) for p in problems]
        caps = capacities or [min(s["nnz_upper"], 4 * s["n_rows"] + 1024) for s in sizes]
        self._create(caps, pool_entries)

    def _create(self, caps, pool_entries):
        d = self.pl.device
        self.models = [self.pl.alloc_model(p, c) for p, c in zip(self.problems, caps)]
        sizes = [mdp_build_query(p) for p in self.problems]
        self.v = [torch.zeros(s["n_states"], dtype=torch.float64, device=d) for s in sizes]
        self.pi = [torch.zeros(s["n_states"], dtype=torch.int32, device=d) for s in sizes]
        self.pool_entries = pool_entries
        nbytes = mdp_batch_query(self.problems, pool_entries)
        self.scratch = torch.empty(nbytes, dtype=torch.uint8, device=d)
        n = self.n
        probs = (MdpProblem * n)(*[problem_struct(p) for p in self.problems])
        envs = (MdpEnv * n)(*[MdpEnv(*[_ptr(e.get(k)) for k, _ in MdpEnv._fields_]) for e in self.envs])
        mods = (MdpModel * n)(*[_model_struct(m) for m in self.models])
        miss = (C.c_int32 * n)(*self.missions)
        vptr = (C.c_void_p * n)(*[t.data_ptr() for t in self.v])
        pptr = (C.c_void_p * n)(*[t.data_ptr() for t in self.pi])
        h = C.c_void_p()
        rc = load().mdp_batch_create(self.pl.ctx, n, probs, envs, mods, miss, vptr, pptr, pool_entries,
                                     self.scratch.data_ptr(), self.scratch.numel(), C.byref(h))
        _check(self.pl.ctx, rc, "mdp_batch_create")
        self.h = h

    def build(self, stream=None):
        _check(self.pl.ctx, load().mdp_batch_build(self.h, _stream_handle(stream)), "mdp_batch_build")

    def solve(self, tol: float = 1e-6, max_sweeps: int = 100000, stream=None):
        _check(self.pl.ctx, load().mdp_batch_solve(self.h, tol, max_sweeps, _stream_handle(stream)),
               "mdp_batch_solve")

    def capture(self, tol: float = 1e-6, max_sweeps: int = 100000, stream=None):
        _check(self.pl.ctx, load().mdp_batch_capture(self.h, tol, max_sweeps, _stream_handle(stream)),
               "mdp_batch_capture")

    def replay(self, stream=None):
        _check(self.pl.ctx, load().mdp_batch_replay(self.h, _stream_handle(stream)), "mdp_batch_replay")

    def stats(self):
        """Per-problem build and solve stats (call after the stream has finished)."""
        b = (MdpBuildStats * self.n)()
        v = (MdpViStats * self.n)()
        _check(self.pl.ctx, load().mdp_batch_stats(self.h, b, v), "mdp_batch_stats")
        conv = lambda s, cls: {k: getattr(s, k) for k, _ in cls._fields_}
        return [conv(x, MdpBuildStats) for x in b], [conv(x, MdpViStats) for x in v]

    def build_checked(self, stream=None):
        """Build; if a model or the staging pool was too small, recreate with exact sizes and
        build again. Returns the per-problem build stats."""
        for _ in range(2):
            self.build(stream)
            (stream or torch.cuda.current_stream()).synchronize()
            bs, _ = self.stats()
            statuses = {s["status"] for s in bs}
            if statuses <= {MDP_OK}:
                return bs
            if statuses - {MDP_OK, MDP_E_CAPACITY, MDP_E_SCRATCH}:
                return bs
            caps = [max(s["nnz"], m["col"].numel()) for s, m in zip(bs, self.models)]
            pool = sum(s["nnz"] for s in bs) + 1024
            self.close()
            self._create(caps, max(pool, self.pool_entries))
        return bs

    def close(self):
        if self.h is not None:
            load().mdp_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mdp_server_footprint(problem: dict) -> int:
    n = C.c_size_t()
    rc = load().mdp_server_footprint(C.byref(problem_struct(problem)), C.byref(n))
    if rc != MDP_OK:
        raise MdpError(rc, "mdp_server_footprint")
    return n.value


class Server:
    """Continuous-batching planner (include/mdp.h, mdp_server_*): requests are
    queued with submit(), each step() admits, builds, sweeps and retires, and
    poll() returns completion records. The model pool is one torch allocation;
    each request's policy (and optionally values) is copied into pinned host
    tensors owned here until its completion is polled."""

    def __init__(self, planner: "Planner", pool_bytes: int, max_inflight: int = 64, sweeps_per_step: int = 8,
                 tol: float = 1e-6, max_sweeps: int = 100000, stream=None, build_share: int = 100,
                 chunk_cost: float = 0.0, large_cost: float = 0.0):
        self.pl = planner
        self.h = None
        self.pool = torch.empty(pool_bytes, dtype=torch.uint8, device=planner.device)
        cfg = MdpServerConfig(max_inflight, sweeps_per_step, max_sweeps, build_share, tol, chunk_cost, large_cost)
        h = C.c_void_p()
        _check(planner.ctx, load().mdp_server_create(planner.ctx, C.byref(cfg), self.pool.data_ptr(),
                                                      self.pool.numel(), C.byref(h)), "mdp_server_create")
        self.h = h
        self.stream = stream
        self.pending = {}  # tag -> (problem, env, pi, v) kept alive until polled

    def submit(self, tag: int, problem: dict, env: dict, mission: int, keep_values: bool = False):
        ns = problem["nt"] * problem["nx"] * problem["ny"]
        pi = torch.empty(ns, dtype=torch.int32, pin_memory=True)
        v = torch.empty(ns, dtype=torch.float64, pin_memory=True) if keep_values else None
        ps = problem_struct(problem)
        es = MdpEnv(*[_ptr(env.get(k)) for k, _ in MdpEnv._fields_])
        rc = load().mdp_server_submit(self.h, C.byref(ps), C.byref(es), mission, pi.data_ptr(),
                                      v.data_ptr() if v is not None else None, tag)
        _check(self.pl.ctx, rc, "mdp_server_submit")
        self.pending[tag] = (problem, env, pi, v)

    def step(self) -> int:
        n = C.c_int32()
        _check(self.pl.ctx, load().mdp_server_step(self.h, _stream_handle(self.stream), C.byref(n)),
               "mdp_server_step")
        return n.value

    def poll(self) -> list:
        """Completion records as dicts, with the policy ("pi") and values ("v") tensors."""
        out = []
        buf = (MdpServed * 64)()
        while True:
            n = C.c_int32()
            _check(self.pl.ctx, load().mdp_server_poll(self.h, buf, 64, C.byref(n)), "mdp_server_poll")
            for k in range(n.value):
                rec = {f: getattr(buf[k], f) for f, _ in MdpServed._fields_ if f != "pad"}
                _, _, pi, v = self.pending.pop(rec["tag"])
                rec["pi"], rec["v"] = pi, v
                out.append(rec)
            if n.value < 64:
                return out

    def info(self) -> dict:
        st = MdpServerState()
        _check(self.pl.ctx, load().mdp_server_info(self.h, C.byref(st)), "mdp_server_info")
        return {f: getattr(st, f) for f, _ in MdpServerState._fields_ if f != "pad"}

    def close(self):
        if self.h is not None:
            load().mdp_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mdp_autotune(ctx, problem: dict, env: dict, stream=None) -> dict:
    """Time every build launch shape on a sample of the problem's first layers and keep
    the fastest on the context for the problem's shape class (waits for the device)."""
    ps = problem_struct(problem)
    n = C.c_size_t()
    rc = load().mdp_autotune_query(C.byref(ps), C.byref(n))
    if rc != MDP_OK:
        raise MdpError(rc, "mdp_autotune_query")
    scratch = torch.empty(n.value, dtype=torch.uint8, device="cuda")
    es = MdpEnv(*[_ptr(env.get(k)) for k, _ in MdpEnv._fields_])
    rep = MdpTuneReport()
    rc = load().mdp_autotune(ctx, C.byref(ps), C.byref(es), scratch.data_ptr(), scratch.numel(), C.byref(rep),
                             _stream_handle(stream))
    _check(ctx, rc, "mdp_autotune")
    k = rep.n_candidates
    shapes = [dict(row_lanes=rep.row_lanes[i], rch=rep.rch[i], pack16=rep.pack16[i], ms=rep.ms[i]) for i in range(k)]
    return dict(best=rep.best, default=rep.default_shape, sample_layers=rep.sample_layers, shapes=shapes)


def mdp_ctx_set_plan(ctx, problem: dict, row_lanes: int, rch: int, pack16: int) -> None:
    """Use this build launch shape for the problem's shape class (row_lanes = 0: default)."""
    rc = load().mdp_ctx_set_plan(ctx, C.byref(problem_struct(problem)), row_lanes, rch, pack16)
    _check(ctx, rc, "mdp_ctx_set_plan")
