"""Batched build + solve (one persistent build launch, one sweep launch per
iteration, optionally replayed from a HIP graph) against the plain
single-problem path, problem by problem (needs an MI355X)."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_2109_00857_amd import workloads as W

from gpu_helpers import assert_matches_oracle, model_to_host

pytestmark = pytest.mark.gpu


def _uneven_problems():
    """Problems of uneven grid, horizon, modes, realizations, headings, sub-grid
    and mission (the kinds of variation of the batched workload, scaled down)."""
    ws = []
    ws.append(W.config1(nt=5, n_real=300, sub_h=3))
    ws.append(W.config2(nx=23, ny=17, nt=4, n_real=700, K=6, n_head=12, missions=(0, 2)))
    ws.append(W.config3(nx=19, ny=21, nt=3, n_real=450, missions=(1, 2)))
    for nx, nt, nr, nh, m in ((24, 3, 200, 9, 2), (29, 4, 350, 13, 0), (34, 5, 500, 16, 1), (39, 6, 650, 11, 2)):
        w = W.config1(nx=nx, ny=nx, nt=nt, n_real=nr, n_head=nh, sub_h=4)
        w.problem["mission_mask"] = 1 << m
        if m == W.MISSION_NET_ENERGY:
            w.gbar = W._gaussian_bump(nx, nx, nt)
        ws.append(w)
    ws[1].problem["flags"] |= 1  # near-edge counting on one problem
    return ws


@pytest.fixture(scope="module")
def planner():
    import torch

    assert torch.cuda.is_available()
    from paper_2109_00857_amd import mdp

    pl = mdp.Planner(0)
    yield pl
    pl.close()


def _plain(planner, w, mission):
    model, stats = planner.build(w.problem, planner.upload_env(w))
    v, vst = planner.value_iterate(w.problem, model, mission)
    pi = planner.policy(w.problem, model, mission, v)
    return model, stats, v, vst, pi


def _same(a, b):
    return a.contiguous().view(-1).cpu().numpy().tobytes() == b.contiguous().view(-1).cpu().numpy().tobytes()


def _check_against_oracle(ora, ws, missions, batch, bstats):
    """Every problem of the batch against the CPU oracle (not only the plain path)."""
    for i, (w, m) in enumerate(zip(ws, missions)):
        print(f"[batch] oracle check of problem {i}: {w.problem['nx']}x{w.problem['ny']}x{w.problem['nt']}",
              flush=True)
        g = model_to_host(batch.models[i], bstats[i])
        assert_matches_oracle(ora, w, [m], g, bstats[i], {m: batch.v[i].cpu().numpy()},
                              {m: batch.pi[i].cpu().numpy()})


def _check_against_plain(planner, ws, missions, batch, bstats, vstats):
    for i, (w, m) in enumerate(zip(ws, missions)):
        model, stats, v, vst, pi = _plain(planner, w, m)
        nnz = stats["nnz"]
        assert bstats[i]["status"] == 0, (i, bstats[i])
        for k in ("nnz", "samples", "n_escape", "n_near_edge"):
            assert bstats[i][k] == stats[k], (i, k, bstats[i][k], stats[k])
        bm = batch.models[i]
        assert _same(bm["row_ptr"], model["row_ptr"]), i
        assert _same(bm["col"][:nnz], model["col"][:nnz]), i
        assert _same(bm["cnt"][:nnz], model["cnt"][:nnz]), i
        assert _same(bm["reward"], model["reward"]), i
        assert vstats[i]["sweeps"] == vst["sweeps"] and vstats[i]["status"] == vst["status"], (i, vstats[i], vst)
        assert _same(batch.v[i], v), i
        assert _same(batch.pi[i], pi), i


def test_batch_equals_plain(planner, ora):
    from paper_2109_00857_amd import mdp

    ws = _uneven_problems()
    missions = [w.missions()[-1] for w in ws]
    envs = [planner.upload_env(w) for w in ws]
    print(f"[batch] {len(ws)} problems, rows {[w.n_rows for w in ws]}", flush=True)
    b = mdp.Batch(planner, [w.problem for w in ws], envs, missions)
    bstats = b.build_checked()
    b.solve()
    import torch

    torch.cuda.synchronize()
    bstats, vstats = b.stats()
    _check_against_plain(planner, ws, missions, b, bstats, vstats)
    _check_against_oracle(ora, ws, missions, b, bstats)
    b.close()


def test_batch_pool_too_small_recovers(planner):
    """A staging pool far too small is reported (MDP_E_SCRATCH) and the binding
    recreates the batch with the exact size."""
    from paper_2109_00857_amd import mdp
    import torch

    ws = _uneven_problems()[:3]
    missions = [w.missions()[0] for w in ws]
    envs = [planner.upload_env(w) for w in ws]
    b = mdp.Batch(planner, [w.problem for w in ws], envs, missions, pool_entries=1000)
    b.build()
    torch.cuda.synchronize()
    first, _ = b.stats()
    assert any(s["status"] == mdp.MDP_E_SCRATCH for s in first)
    bstats = b.build_checked()
    assert all(s["status"] == 0 for s in bstats), bstats
    b.solve()
    torch.cuda.synchronize()
    bstats, vstats = b.stats()
    _check_against_plain(planner, ws, missions, b, bstats, vstats)
    b.close()


def test_batch_graph_replays(planner):
    """Build + solve captured once and replayed several times, with eager work and
    synchronisations between replays: every replay gives the eager result."""
    from paper_2109_00857_amd import mdp
    import torch

    ws = _uneven_problems()[2:6]
    missions = [w.missions()[-1] for w in ws]
    envs = [planner.upload_env(w) for w in ws]
    b = mdp.Batch(planner, [w.problem for w in ws], envs, missions)
    b.build_checked()
    b.solve()
    torch.cuda.synchronize()
    nnz = [s["nnz"] for s in b.stats()[0]]
    ref_sweeps = [s["sweeps"] for s in b.stats()[1]]
    ref_models = [{k: t.clone() for k, t in m.items()} for m in b.models]
    ref_v = [t.clone() for t in b.v]
    ref_pi = [t.clone() for t in b.pi]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.capture(stream=s)
    s.synchronize()
    for rep in range(3):
        for m in b.models:  # scribble over the outputs so each replay must rewrite them
            m["col"].fill_(-1)
            m["reward"].fill_(float("nan"))
        for t in b.v:
            t.fill_(123.0)
        torch.cuda.synchronize()
        b.replay(stream=s)
        s.synchronize()
        _ = torch.ones(1024, device=planner.device).sum().item()  # eager work between replays
        bs, vs = b.stats()
        assert all(x["status"] == 0 for x in bs) and all(x["status"] == 0 for x in vs), (rep, bs, vs)
        # every replay starts cold: the same sweep counts as the eager solve
        assert [x["sweeps"] for x in vs] == ref_sweeps, (rep, vs)
        for i in range(len(ws)):
            for k in ("row_ptr", "reward"):
                assert _same(b.models[i][k], ref_models[i][k]), (rep, i, k)
            for k in ("col", "cnt"):  # entries past nnz are capacity slack, never written
                assert _same(b.models[i][k][:nnz[i]], ref_models[i][k][:nnz[i]]), (rep, i, k)
            assert _same(b.v[i], ref_v[i]), (rep, i)
            assert _same(b.pi[i], ref_pi[i]), (rep, i)
    b.close()


def _sampled_rows_and_bellman(ora, w, m, model, v, pi, rng, n_rows=12, n_states=4):
    """Sampled rows bit-exact against the oracle's rows, and at sampled states one
    Bellman step with the oracle's rows and the GPU's next-layer values gives the
    GPU's value, the GPU's action attaining the maximum (both within 1e-5 of the
    state's absolute scale)."""
    import torch

    p = w.problem
    nc, na, ns, nr = p["nx"] * p["ny"], w.n_actions, w.n_states, p["n_real"]
    rows = np.sort(rng.choice(w.n_rows, n_rows, replace=False))
    rp = model["row_ptr"][torch.as_tensor(np.concatenate([rows, rows + 1]), device=model["row_ptr"].device)]
    rp = rp.cpu().numpy()
    R = model["reward"][0, torch.as_tensor(rows, device=model["reward"].device)].cpu().numpy().astype(np.float64)
    for k, row in enumerate(rows):
        s, a = divmod(int(row), na)
        t, c = divmod(s, nc)
        cols, cnts, Ro, Ao, ne, _ = ora.row(w, t, c, a)
        assert ne == 0
        lo, hi = rp[k], rp[len(rows) + k]
        np.testing.assert_array_equal(model["col"][lo:hi].cpu().numpy(), cols, err_msg=f"row {row}")
        np.testing.assert_array_equal(model["cnt"][lo:hi].cpu().numpy().astype(np.int32), cnts, err_msg=f"row {row}")
        assert abs(R[k] - Ro[m]) <= 1e-5 * Ao[m], (row, R[k], Ro[m], Ao[m])
    for s in rng.choice(ns, n_states, replace=False):
        t, c = divmod(int(s), nc)
        q = np.zeros(na)
        scale = 0.0
        for a in range(na):
            cols, cnts, Ro, Ao, _, _ = ora.row(w, t, c, a)
            tr = cols < ns
            q[a] = Ro[m] + float((cnts[tr] * v[cols[tr]]).sum()) / nr
            scale = max(scale, Ao[m] + float((cnts[tr] * np.abs(v[cols[tr]])).sum()) / nr)
        assert abs(v[s] - q.max()) <= 1e-5 * scale, (int(s), v[s], q.max(), scale)
        assert q[pi[s]] >= q.max() - 1e-5 * scale, (int(s), pi[s], q[pi[s]], q.max())


def test_batched_mix_against_oracle(planner, ora):
    """The 64-instance uneven batch as benchmarked (sub-grids sized on the device,
    one persistent build per kernel group, one sweep launch per iteration): the
    four smallest instances whole against the oracle; every instance on sampled
    rows (bit-exact counts) and on the Bellman identity at sampled states."""
    import torch

    from paper_2109_00857_amd import mdp

    ws = [W.batched_instance(i) for i in range(64)]
    envs = [planner.upload_env(w) for w in ws]
    for w, env in zip(ws, envs):
        w.problem["sub_hx"], w.problem["sub_hy"] = mdp.mdp_subgrid_auto(planner.ctx, w.problem, env)
    missions = [w.missions()[0] for w in ws]
    print(f"[batch] 64-instance mix: {sum(w.nominal_samples for w in ws):.3e} samples", flush=True)
    # the oracle's whole models of the four smallest instances, built on host
    # threads (the C oracle runs without the GIL) while the GPU works
    order = np.argsort([w.nominal_samples for w in ws])
    smallest = [int(i) for i in order[:4]]
    pool = ThreadPoolExecutor(max_workers=4)
    futs = {i: pool.submit(ora.build_model, ws[i]) for i in smallest}
    b = mdp.Batch(planner, [w.problem for w in ws], envs, missions)
    bstats = b.build_checked()
    assert all(s["status"] == 0 for s in bstats), bstats
    b.solve()
    torch.cuda.synchronize()
    bstats, vstats = b.stats()
    assert all(s["status"] == 0 for s in vstats), vstats
    for i in smallest:
        w, m = ws[i], missions[i]
        print(f"[batch] instance {i} whole against the oracle ({w.nominal_samples:.2e} samples)", flush=True)
        g = model_to_host(b.models[i], bstats[i])
        assert_matches_oracle(ora, w, [m], g, bstats[i], {m: b.v[i].cpu().numpy()}, {m: b.pi[i].cpu().numpy()},
                              om=futs[i].result())
    pool.shutdown()
    rng = np.random.default_rng(77)
    for i, (w, m) in enumerate(zip(ws, missions)):
        _sampled_rows_and_bellman(ora, w, m, b.models[i], b.v[i].cpu().numpy(), b.pi[i].cpu().numpy(), rng)
    print("[batch] 64 instances: sampled rows and states match the oracle", flush=True)
    b.close()
