"""Incremental re-planning (mdp_build_from + mdp_value_iterate_layers) against
a full rebuild and solve on the new environment and against the oracle
(needs an MI355X)."""
import numpy as np
import pytest

from paper_2109_00857_amd import workloads as W

from gpu_helpers import assert_counts_equal, assert_rewards_close, model_to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def planner():
    import torch

    assert torch.cuda.is_available()
    from paper_2109_00857_amd import mdp

    pl = mdp.Planner(0)
    yield pl
    pl.close()


def _same(a, b):
    return a.contiguous().view(-1).cpu().numpy().tobytes() == b.contiguous().view(-1).cpu().numpy().tobytes()


def _updated(w, t0, seed):
    """The same problem after a forecast update at layer t0: new coefficient
    draws for layers >= t0 (the earlier layers keep theirs)."""
    w2 = W.Workload(w.name, dict(w.problem), w.ubar, w.vbar, w.phiu, w.phiv, w.mu.copy(), w.gbar, w.mask)
    rng = np.random.default_rng(seed)
    K, nr = w.mu.shape[1], w.mu.shape[2]
    sig = (0.2 / np.arange(1, K + 1))[:, None]
    w2.mu[t0:] = (1.3 * sig * rng.standard_normal((w.mu.shape[0] - t0, K, nr))).astype(np.float32)
    return w2


@pytest.mark.parametrize("t0", [1, 4, 6])
def test_build_from_equals_full_rebuild(planner, ora, t0):
    import torch

    from paper_2109_00857_amd import mdp

    w = W.config2(nx=31, ny=27, nt=7, n_real=900)
    w2 = _updated(w, t0, 100 + t0)
    p = w.problem
    env, env2 = planner.upload_env(w), planner.upload_env(w2)
    print(f"[replan] t0={t0}", flush=True)
    ref, ref_st = planner.build(p, env2)  # full build on the new environment
    assert ref_st["status"] == 0
    old = planner.alloc_model(p, ref_st["nnz"] + 5000, packed=True)  # room for the rebuilt model
    scratch = planner.scratch(p)
    st = mdp.stats_buffer(mdp.MdpBuildStats)
    mdp.mdp_build(planner.ctx, p, env, old, scratch, st)
    assert mdp.mdp_build_sync(planner.ctx, st) == mdp.MDP_OK
    mdp.mdp_build_from(planner.ctx, p, env2, old, t0, scratch, st)
    assert mdp.mdp_build_sync(planner.ctx, st) == mdp.MDP_OK
    s = mdp.read_stats(st, mdp.MdpBuildStats)
    nnz = ref_st["nnz"]
    assert s["nnz"] == nnz
    nc, na = p["nx"] * p["ny"], w.n_actions
    rows_rebuilt = (p["nt"] - t0) * nc * na
    assert s["samples"] < ref_st["samples"] and s["samples"] <= rows_rebuilt * p["n_real"]
    assert _same(old["row_ptr"], ref["row_ptr"]) and _same(old["reward"], ref["reward"])
    assert _same(old["col"][:nnz], ref["col"][:nnz]) and _same(old["cnt"][:nnz], ref["cnt"][:nnz])
    assert _same(old["ent"][:nnz], ref["ent"][:nnz])  # the fused sweep's packed entries too
    assert _same(old["roff"], ref["roff"])
    # and the rebuilt model is the oracle's model of the new environment
    om = ora.build_model(w2)
    g = model_to_host(old, s)
    assert_counts_equal(g, om)
    assert_rewards_close(g, om, w2.missions())

    # values of layers >= t0 from the layer-restricted solve (warm start from the
    # old model's values) equal the full solve on the new model, bit for bit
    for m in w.missions():
        v_full, vst_full = planner.value_iterate(p, ref, m)
        v_old, _ = planner.value_iterate(p, ref, m)  # any v0: take a converged vector and perturb it
        v0 = v_old.clone()
        v0[t0 * nc:] += 3.0
        v = v0.clone()
        vsc = planner.scratch(p)
        vst = mdp.stats_buffer(mdp.MdpViStats)
        mdp.mdp_value_iterate_layers(planner.ctx, p, old, m, t0, 1e-6, 100000, v, vsc, vst)
        torch.cuda.synchronize()
        vs = mdp.read_stats(vst, mdp.MdpViStats)
        assert vs["status"] == 0 and vs["sweeps"] <= p["nt"] - t0 + 1, vs
        assert _same(v[t0 * nc:], v_full[t0 * nc:]), m
        assert _same(v[: t0 * nc], v0[: t0 * nc]), m  # earlier layers untouched
        pi_full = planner.policy(p, ref, m, v_full)
        pi = planner.policy(p, old, m, v)
        assert _same(pi[t0 * nc:], pi_full[t0 * nc:]), m


def test_build_from_capacity_and_arguments(planner):
    from paper_2109_00857_amd import mdp

    # a sub-grid wide enough for three times the spread (7 x 4 half widths needed)
    w = W.config1(nt=5, n_real=200, sub_h=7)
    p = w.problem
    env = planner.upload_env(w)
    model, st0 = planner.build(p, env)
    assert st0["status"] == 0
    w2 = _updated(w, 2, 9)
    w2.mu[2:] *= 3.0  # a wider spread: more nonzeros in the rebuilt layers
    env2 = planner.upload_env(w2)
    ref, ref_st = planner.build(p, env2)
    scratch = planner.scratch(p)
    st = mdp.stats_buffer(mdp.MdpBuildStats)
    small = {k: v for k, v in model.items()}
    assert ref_st["status"] == 0 and ref_st["nnz"] > st0["nnz"], (ref_st, st0)
    if ref_st["nnz"] > st0["nnz"]:  # the current capacity (st0 nnz) is too small for the new model
        mdp.mdp_build_from(planner.ctx, p, env2, small, 2, scratch, st)
        assert mdp.mdp_build_sync(planner.ctx, st) == mdp.MDP_E_CAPACITY
        assert mdp.read_stats(st, mdp.MdpBuildStats)["nnz"] == ref_st["nnz"]
    for bad in (-1, p["nt"]):
        with pytest.raises(mdp.MdpError):
            mdp.mdp_build_from(planner.ctx, p, env2, model, bad, scratch, st)
    v = __import__("torch").zeros(w.n_states, dtype=__import__("torch").float64, device=planner.device)
    with pytest.raises(mdp.MdpError):
        mdp.mdp_value_iterate_layers(planner.ctx, p, model, 0, p["nt"], 1e-6, 10, v, scratch,
                                     mdp.stats_buffer(mdp.MdpViStats))
