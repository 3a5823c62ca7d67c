"""The allocation-free value iteration (mdp_value_iterate_noalloc: the
library's static per-GPU scratch instead of a caller buffer) against
mdp_value_iterate with a caller scratch, through the C ABI: the same values and
stats bit for bit on two calls in a row, the first on the 200 x 200 x 200
instance (8 million states, near the scratch's limit), the second on a smaller
problem; problems beyond the static scratch are refused on the host."""
import numpy as np
import pytest

from paper_2109_00857_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def planner():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("needs an MI355X")
    from paper_2109_00857_amd import mdp

    pl = mdp.Planner(0)
    yield pl
    pl.close()


def _both(pl, w, mission):
    import torch

    from paper_2109_00857_amd import mdp

    p = dict(w.problem)
    env = pl.upload_env(w)
    if p["sub_hx"] == 0 and p["sub_hy"] == 0:  # sub-grid sized from the flow
        p["sub_hx"], p["sub_hy"] = mdp.mdp_subgrid_auto(pl.ctx, p, env)
    model, st = pl.build(p, env)
    assert st["status"] == mdp.MDP_OK, st
    ns = mdp.mdp_build_query(p)["n_states"]
    assert 8 * ns < mdp.MDP_NOALLOC_SCRATCH_BYTES
    s = torch.cuda.current_stream()
    # the existing entry point, on a caller scratch filled with garbage
    scratch = pl.scratch(p)
    scratch.fill_(0xA5)
    v_ref = torch.zeros(ns, dtype=torch.float64, device=pl.device)
    st_ref = mdp.stats_buffer(mdp.MdpViStats)
    mdp.mdp_value_iterate(pl.ctx, p, model, mission, 1e-6, 100000, v_ref, scratch, st_ref, s)
    # the allocation-free one
    v = torch.zeros(ns, dtype=torch.float64, device=pl.device)
    st_na = mdp.stats_buffer(mdp.MdpViStats)
    mdp.mdp_value_iterate_noalloc(pl.ctx, p, model, mission, 1e-6, 100000, v, st_na, s)
    s.synchronize()
    a, b = mdp.read_stats(st_ref, mdp.MdpViStats), mdp.read_stats(st_na, mdp.MdpViStats)
    assert a["status"] == mdp.MDP_OK and a == b, (a, b)
    assert torch.equal(v, v_ref)
    assert torch.isfinite(v).all()
    return a


def test_noalloc_equals_scratch_path(planner):
    print("[noalloc] 200x200x200 instance, net-energy mission", flush=True)
    big = W.config3()
    s1 = _both(planner, big, W.MISSION_NET_ENERGY)
    assert s1["sweeps"] >= 2
    del big
    print("[noalloc] then the 25x25x20 instance", flush=True)
    s2 = _both(planner, W.config1(), W.MISSION_TIME)
    assert 2 <= s2["sweeps"] <= 21


def test_noalloc_refuses_problems_above_its_scratch(planner):
    import torch

    from paper_2109_00857_amd import mdp

    w = W.config1(nt=2, n_real=50, sub_h=3)
    p = dict(w.problem)
    model, st = planner.build(p, planner.upload_env(w))
    assert st["status"] == mdp.MDP_OK
    big = dict(p, nx=1000, ny=1000, nt=10)  # 1e7 states: 80 MB of values, refused before any device work
    v = torch.zeros(16, dtype=torch.float64, device=planner.device)
    with pytest.raises(mdp.MdpError) as e:
        mdp.mdp_value_iterate_noalloc(planner.ctx, big, model, 0, 1e-6, 10, v, mdp.stats_buffer(mdp.MdpViStats))
    assert e.value.status == mdp.MDP_E_SCRATCH
