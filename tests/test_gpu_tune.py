"""Autotuner on the GPU: every candidate launch configuration (lanes 4-32,
team sizes, grid sizes) must reproduce the default configuration's results,
and the cached choice must be picked up by later calls."""

import numpy as np
import pytest

from oracle import oracle as O
from paper_1705_02403_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1705_02403_amd import gmt


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    gmt.use_torch_allocator()
    gmt.gmt_tune_clear()
    yield
    gmt.gmt_tune_clear()


def eu_queries(seeds, lam=0.5):
    rms, qs, probs = [], [], []
    for seed in seeds:
        p = I.problem_2d(seed, lam=lam)
        rm = gmt.gmt_build_neighbors(torch.from_numpy(p.samples).cuda(), gmt.GMT_COST_EUCLIDEAN,
                                     O.euclid_radius(p))
        rms.append(rm)
        probs.append(p)
        qs.append(gmt.BatchQuery(rm, p.x_init, gmt.make_goal(p.goal_center, p.goal_radius, 2), p.boxes, p.lam))
    return rms, qs, probs


def test_batch_tuning_keeps_results(setup):
    say("tune: 2D batch")
    rms, qs, probs = eu_queries(range(8))
    opts = gmt.make_opts(edge_step=0.005)
    ref = gmt.gmt_plan_batch(qs, gmt.make_opts(edge_step=0.005, lanes=16, team_wgs=1))
    ch = gmt.gmt_autotune(qs, opts, single=False, reps=1)
    assert ch["candidates"] == 36 and ch["lanes"] in (4, 8, 16, 32) and ch["team_wgs"] in (1, 2, 4)
    assert ch["threads"] in (256, 512, 1024)
    assert ch["ms"] <= ch["default_ms"]
    hit = gmt.gmt_tune_lookup(gmt.tune_shape(gmt.GMT_COST_EUCLIDEAN, 2, 2000, 20, 8))
    assert (hit["lanes"], hit["team_wgs"], hit["workgroups"], hit["threads"]) == \
        (ch["lanes"], ch["team_wgs"], ch["workgroups"], ch["threads"])
    got = gmt.gmt_plan_batch(qs, opts)  # knobs at 0: the tuned choice
    for a, b in zip(got, ref):
        assert a.status == b.status and a.path_cost == b.path_cost and list(a.path) == list(b.path)
    for rm in rms:
        rm.free()


def test_single_tuning_double_integrator(setup):
    say("tune: DI single plan")
    s = I.di_samples(1, 4096)
    r = 1.75 * 4.0 ** (1.0 / 6.0)
    rm = gmt.gmt_build_neighbors(torch.from_numpy(s).cuda(), gmt.GMT_COST_DOUBLE_INTEGRATOR, r)
    p = I.di_problem(3, s, r=r, sample_seed=1)
    q = gmt.BatchQuery(rm, p.x_init, gmt.make_goal(p.goal_center, p.goal_radius, 3), p.boxes, p.lam)
    opts = gmt.make_opts(traj_points=16)
    ch = gmt.gmt_autotune([q], opts, single=True, reps=1)
    assert ch["candidates"] >= 16 and ch["lanes"] in (4, 8, 16, 32) and ch["team_wgs"] >= 1
    alone = gmt.gmt_plan(rm, p.x_init, q.goal, p.boxes, p.lam, gmt.make_opts(traj_points=16, lanes=16, threads=256),
                         outputs=False)
    tuned = gmt.gmt_plan(rm, p.x_init, q.goal, p.boxes, p.lam, opts, outputs=False)
    assert tuned.status == alone.status and tuned.path_cost == alone.path_cost
    assert list(tuned.path) == list(alone.path)
    rm.free()


@pytest.mark.parametrize("lanes", [4, 32])
def test_new_lane_widths_match_oracle(setup, lanes):
    say("tune: lanes %d vs oracle" % lanes)
    rms, qs, probs = eu_queries([5, 6], lam=0.2)
    out = gmt.gmt_plan_batch(qs, gmt.make_opts(edge_step=0.005, lanes=lanes))
    for p, o in zip(probs, out):
        ref = O.plan(p, O.euclid_radius(p), O.neighbors(p.samples, O.EUCLID, O.euclid_radius(p)))
        assert o.status == ref.status
        if ref.status == O.OK:
            assert o.path_cost == ref.path_cost and list(o.path) == list(ref.path)
    for rm in rms:
        rm.free()
