"""Continuous-batching server (mdp_server_*) against the plain single-problem
path, request by request (needs an MI355X)."""
import pytest

from paper_2109_00857_amd import workloads as W

from gpu_helpers import assert_policy_optimal, assert_values_close

pytestmark = pytest.mark.gpu


def _requests():
    """Uneven requests: grid, horizon, modes, realizations, headings, sub-grid,
    mission, and one with near-edge counting."""
    out = []
    for k, (nx, nt, nr, nh) in enumerate(((14, 4, 300, 8), (25, 9, 500, 12), (18, 3, 250, 9), (31, 6, 420, 16),
                                           (22, 12, 350, 10), (27, 5, 650, 13))):
        w = W.config1(nx=nx, ny=nx, nt=nt, n_real=nr, n_head=nh, sub_h=3 + k % 2, seed=k)
        m = k % 3
        if m == W.MISSION_NET_ENERGY:
            w.gbar = W._gaussian_bump(nx, nx, nt)
        out.append((w, m))
    w = W.config2(nx=21, ny=19, nt=7, n_real=600, K=6, n_head=12, missions=(1,))
    w.problem["flags"] |= 1
    out.append((w, 1))
    return out


@pytest.fixture(scope="module")
def planner():
    import torch

    assert torch.cuda.is_available()
    from paper_2109_00857_amd import mdp

    pl = mdp.Planner(0)
    yield pl
    pl.close()


def _plain(planner, w, m):
    p = dict(w.problem)
    p["mission_mask"] = 1 << m
    model, stats = planner.build(p, planner.upload_env(w))
    v, vst = planner.value_iterate(p, model, m)
    pi = planner.policy(p, model, m, v)
    return stats, v.cpu(), vst, pi.cpu()


def _run(srv, reqs, envs, per_step=2):
    """Submit per_step requests before each step until all are queued, then step to the end."""
    done, k, steps = {}, 0, 0
    while len(done) < len(reqs):
        for _ in range(per_step):
            if k < len(reqs):
                w, m = reqs[k]
                srv.submit(k, w.problem, envs[k], m, keep_values=True)
                k += 1
        srv.step()
        steps += 1
        assert steps < 10000
        for rec in srv.poll():
            done[rec["tag"]] = rec
    return done


def _check_oracle(ora, reqs, done):
    """Every served request's values and policy against the CPU oracle."""
    for tag, (w, m) in enumerate(reqs):
        rec = done[tag]
        w1 = W.Workload(w.name, dict(w.problem, mission_mask=1 << m), w.ubar, w.vbar, w.phiu, w.phiv, w.mu,
                        w.gbar, w.mask)
        om = ora.build_model(w1)
        assert rec["nnz"] == om["nnz"], (tag, rec["nnz"], om["nnz"])
        v_ora, _, w_ora = ora.backward(w1, om, m)
        assert_values_close(rec["v"].numpy(), v_ora, w_ora)
        assert_policy_optimal(ora, w1, om, m, v_ora, w_ora, rec["pi"].numpy())


def _check(planner, reqs, done):
    for tag, (w, m) in enumerate(reqs):
        rec = done[tag]
        stats, v, vst, pi = _plain(planner, w, m)
        assert rec["status"] == 0 and rec["build_status"] == 0, rec
        assert rec["nnz"] == stats["nnz"] and rec["samples"] == stats["samples"], (tag, rec, stats)
        assert rec["sweeps"] == vst["sweeps"], (tag, rec["sweeps"], vst)
        assert rec["pi"].numpy().tobytes() == pi.numpy().tobytes(), tag
        assert rec["v"].numpy().tobytes() == v.numpy().tobytes(), tag
        p = w.problem
        assert rec["v_start"] == float(v[p["start_j"] * p["nx"] + p["start_i"]]), tag


def test_served_equals_plain(planner, ora):
    from paper_2109_00857_amd import mdp

    reqs = _requests()
    envs = [planner.upload_env(w) for w, _ in reqs]
    srv = mdp.Server(planner, pool_bytes=1 << 30, max_inflight=3, sweeps_per_step=3)
    done = _run(srv, reqs, envs)
    info = srv.info()
    assert info["queued"] == 0 and info["in_flight"] == 0 and info["pool_used"] == 0, info
    _check(planner, reqs, done)
    _check_oracle(ora, reqs, done)
    srv.close()


def test_served_both_lanes_chunked(planner, ora):
    """Small thresholds send the larger requests to the large-build lane and split
    every build batch into several persistent launches of a few tiles each, with
    up to kServeAhead of them in flight per lane and both lanes building at once:
    each result equals its plain solve bit for bit and the oracle's within
    tolerance."""
    from paper_2109_00857_amd import mdp

    reqs = _requests()
    envs = [planner.upload_env(w) for w, _ in reqs]
    costs = sorted(w.n_rows * w.problem["n_real"] for w, _ in reqs)
    large = float(costs[len(costs) // 2])  # about half the requests take the large lane
    srv = mdp.Server(planner, pool_bytes=1 << 30, max_inflight=6, sweeps_per_step=2, chunk_cost=2e6,
                     large_cost=large)
    done = _run(srv, reqs, envs, per_step=4)
    assert srv.info()["pool_used"] == 0
    _check(planner, reqs, done)
    _check_oracle(ora, reqs, done)
    srv.close()


def test_served_small_pool_is_fifo(planner):
    """A pool that holds about one request at a time: admissions wait, in order."""
    from paper_2109_00857_amd import mdp

    reqs = _requests()[:5]
    envs = [planner.upload_env(w) for w, _ in reqs]
    need = max(mdp.mdp_server_footprint(dict(w.problem, mission_mask=1 << m)) for w, m in reqs)
    srv = mdp.Server(planner, pool_bytes=need + (1 << 20), max_inflight=8, sweeps_per_step=5)
    done = _run(srv, reqs, envs, per_step=5)
    admits = [done[t]["admit_step"] for t in range(len(reqs))]
    assert admits == sorted(admits), admits
    assert srv.info()["pool_used"] == 0
    _check(planner, reqs, done)
    srv.close()


def test_served_rejects_oversized(planner):
    from paper_2109_00857_amd import mdp

    w, m = _requests()[1]
    srv = mdp.Server(planner, pool_bytes=1 << 20, max_inflight=2)
    with pytest.raises(mdp.MdpError) as ei:
        srv.submit(0, w.problem, planner.upload_env(w), m)
    assert ei.value.status == mdp.MDP_E_CAPACITY
    srv.close()
