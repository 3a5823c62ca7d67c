"""Build launch shapes (lane mapping / cell tile, realization chunk, counter
width) change speed only: every shape gives the default shape's model bit for
bit, and the autotuner's choice is used by plain builds and batches (needs an
MI355X)."""
import pytest

from paper_2109_00857_amd import workloads as W

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


def _cases():
    w1 = W.config2(nx=37, ny=29, nt=5, n_real=900)
    w2 = W.config3(nx=23, ny=19, nt=3, n_real=700)
    w3 = W.config1(nt=4, n_real=300, sub_h=3)
    w1.problem["flags"] |= 1
    return [("c2-shaped", w1), ("c3-shaped", w2), ("c1-shaped", w3)]


@pytest.mark.parametrize("case", [0, 1, 2])
def test_every_launch_shape_gives_the_same_model(planner, ora, case):
    from paper_2109_00857_amd import mdp

    from gpu_helpers import assert_counts_equal, assert_rewards_close, model_to_host

    name, w = _cases()[case]
    p = w.problem
    env = planner.upload_env(w)
    mdp.mdp_ctx_set_plan(planner.ctx, p, 0, 0, 0)
    ref, ref_st = planner.build(p, env)
    assert ref_st["status"] == 0
    # the default shape's model is the oracle's (every other shape is compared with it bit for bit)
    om = ora.build_model(w)
    assert ref_st["nnz"] == om["nnz"] and ref_st["n_near_edge"] in (-1, om["n_near_edge"])
    g = model_to_host(ref, ref_st)
    assert_counts_equal(g, om)
    assert_rewards_close(g, om, w.missions())
    rep = mdp.mdp_autotune(planner.ctx, p, env)
    shapes = rep["shapes"]
    print(f"[tune] {name}: {len(shapes)} shapes, best {shapes[rep['best']]}", flush=True)
    assert len(shapes) >= 2 and 0 <= rep["best"] < len(shapes)
    assert all(s["ms"] > 0 for s in shapes)
    for sh in shapes:
        mdp.mdp_ctx_set_plan(planner.ctx, p, sh["row_lanes"], sh["rch"], sh["pack16"])
        m, st = planner.build(p, env)
        for k in ("status", "nnz", "samples", "n_escape", "n_near_edge"):
            assert st[k] == ref_st[k], (sh, k, st[k], ref_st[k])
        for k in ("row_ptr", "col", "cnt", "reward"):
            assert _same(m[k], ref[k]), (sh, k)
    mdp.mdp_ctx_set_plan(planner.ctx, p, 0, 0, 0)


def test_batch_uses_context_shape(planner):
    """A batch on a context with a non-default shape for one problem's class
    equals the plain default build."""
    from paper_2109_00857_amd import mdp
    import torch

    ws = [w for _, w in _cases()]
    missions = [w.missions()[-1] for w in ws]
    envs = [planner.upload_env(w) for w in ws]
    mdp.mdp_ctx_set_plan(planner.ctx, ws[0].problem, 64, 256, 0)
    b = mdp.Batch(planner, [w.problem for w in ws], envs, missions)
    bs = b.build_checked()
    b.solve()
    torch.cuda.synchronize()
    mdp.mdp_ctx_set_plan(planner.ctx, ws[0].problem, 0, 0, 0)
    for i, w in enumerate(ws):
        ref, st = planner.build(w.problem, envs[i])
        assert bs[i]["nnz"] == st["nnz"], i
        for k in ("row_ptr", "reward"):
            assert _same(b.models[i][k], ref[k]), (i, k)
        for k in ("col", "cnt"):
            assert _same(b.models[i][k][: st["nnz"]], ref[k]), (i, k)
